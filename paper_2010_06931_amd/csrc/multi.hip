// More than two volumes (Sec. 2.1 input: at least two raster scans, at least
// one orthogonal to the others).  Every volume V has an orientation o_V (0:
// X-fast, B-scans are rows j; 1: Y-fast, columns i) and its own field d^V.
// The objective is
//   sum over volume pairs P < Q of the two-volume data term (Eqs. 2-9, the
//   pair's own eta, validity resampled along each volume's slow axis)
//   + alpha sum_V R_V (each volume in its own acquisition order)
//   + M = gamma d / (n N_A) sum_c (sum_V sum_ij d^V_ij,c)^2,
// which is the pair objective for n = 2.
//
// Each volume is ingested once (float32 staging, validity, projection or
// depth mean, OCTA substitution, pyramid).  Every volume pair evaluates with
// the pair kernels through a view pair that borrows the two volumes'
// pyramids (alpha / (n - 1) so that each R_V counts once, gamma = 0); the
// pairs' float64 gradients are summed per volume in a fixed order, M is
// added from the fixed-order sum of all fields, and the device L-BFGS of the
// pair solve runs over all n fields.
#include <atomic>
#include <memory>
#include <utility>
#include <vector>

#include "runtime_types.h"

namespace octmc {
namespace {

constexpr int kMB = 256;       // threads per block of the reductions here
constexpr int kMBlocks = 512;  // block partials of the reductions here

size_t esz(octmc_dtype dt) { return dt == OCTMC_F32 ? 4 : 2; }

// device temporaries freed with the list
struct DevBufList {
    std::vector<void*> p;
    ~DevBufList()
    {
        for (void* q : p) (void)hipFree(q);
    }
    void* get(size_t bytes)
    {
        void* q = nullptr;
        if (hipMalloc(&q, bytes ? bytes : 16) != hipSuccess) return nullptr;
        p.push_back(q);
        return q;
    }
};

struct VolumePyr {
    int orient = 0;
    void* s[OCTMC_MAX_LEVELS] = {};   // structural volume, storage type
    float* a[OCTMC_MAX_LEVELS] = {};  // en face image
    float* v[OCTMC_MAX_LEVELS] = {};  // validity (h values for X-fast, w for Y-fast)
    float* octa = nullptr;            // finest OCTA volume, invalid B-scans replaced
};

// sum of all fields per component, block partials then a fixed-order final
// skip (device flag, may be null) on every kernel here: when nonzero the
// launch does nothing (the solver's device form enqueues evaluations ahead)
__global__ __launch_bounds__(kMB) void k_field_sum(const float* __restrict__ disp, size_t nq, double* __restrict__ blk,
                                                   const int* __restrict__ skip)
{
    if (skip && *skip) return;
    __shared__ double red[3][kMB];
    double s[3] = {0.0, 0.0, 0.0};
    for (size_t q = (size_t)blockIdx.x * kMB + threadIdx.x; q < nq; q += (size_t)gridDim.x * kMB)
        for (int c = 0; c < 3; ++c) s[c] += (double)disp[q * 3 + c];
    for (int c = 0; c < 3; ++c) red[c][threadIdx.x] = s[c];
    __syncthreads();
    for (int w = kMB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) blk[(size_t)blockIdx.x * 3 + c] = red[c][0];
}

// lanes sum contiguous runs of partials in order, then a fixed butterfly
__device__ __forceinline__ double wave_sum_rows(const double* __restrict__ blk, int stride, int row, int nblk)
{
    const int lane = threadIdx.x & 63;
    const int per = (nblk + 63) / 64;
    double s = 0.0;
    for (int e = 0; e < per; ++e) {
        const int b = lane * per + e;
        if (b < nblk) s += blk[(size_t)b * stride + row];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    return s;
}

// the three field sums from the block partials of k_field_sum (one wave each)
__global__ __launch_bounds__(kMB) void k_field_sum_final(const double* __restrict__ blk, int nblk,
                                                         double* __restrict__ S, const int* __restrict__ skip)
{
    if (skip && *skip) return;
    const int wv = threadIdx.x >> 6;
    if (wv >= 3) return;  // uniform per wave
    const double s = wave_sum_rows(blk, 3, wv, nblk);
    if ((threadIdx.x & 63) == 0) S[wv] = s;
}

struct GatherSpec {
    const double* pg[kMaxVol * (kMaxVol - 1) / 2];  // per pair gradient [2][na][3]
    signed char pq[kMaxVol][kMaxVol - 1];  // for each volume: its pairs in order
    signed char slot[kMaxVol][kMaxVol - 1];
    int n;
};

// gradient per volume = sum over its pairs (pair order) + dM/dd; g . p partials
__global__ __launch_bounds__(kMB) void k_gather(const GatherSpec spec, size_t na, const double* __restrict__ Sdev,
                                                double mscale, const double* __restrict__ p,
                                                double* __restrict__ g64, float* __restrict__ g32,
                                                double* __restrict__ blk, const int* __restrict__ skip)
{
    if (skip && *skip) return;
    __shared__ double red[kMB];
    const double S[3] = {Sdev[0], Sdev[1], Sdev[2]};
    double gp = 0.0;
    const size_t nr = na * 3;
    for (size_t r = (size_t)blockIdx.x * kMB + threadIdx.x; r < nr; r += (size_t)gridDim.x * kMB) {
        const int c = (int)(r % 3);
        for (int V = 0; V < spec.n; ++V) {
            double g = 0.0;
            for (int t = 0; t < spec.n - 1; ++t)
                g += spec.pg[spec.pq[V][t]][(size_t)spec.slot[V][t] * nr + r];
            g += mscale * S[c];
            const size_t e = (size_t)V * nr + r;
            if (g64) g64[e] = g;
            if (g32) g32[e] = (float)g;
            if (p) gp += g * p[e];
        }
    }
    red[threadIdx.x] = gp;
    __syncthreads();
    for (int w = kMB / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) blk[blockIdx.x] = red[0];
}

struct FinalSpec {
    const double* pt[kMaxVol * (kMaxVol - 1) / 2];  // per pair terms
    int npairs, n, d;
    double gamma, alpha, na;
};

// multi-volume terms from the pairs' terms (pair order), M and g . p; one wave
__global__ __launch_bounds__(64) void k_multi_final(const FinalSpec spec, const double* __restrict__ Sdev,
                                                    const double* __restrict__ gp_blk, int ngp,
                                                    double* __restrict__ terms, const int* __restrict__ skip)
{
    if (skip && *skip) return;
    const double gp = wave_sum_rows(gp_blk, 1, 0, ngp);
    if (threadIdx.x != 0) return;
    const double S[3] = {Sdev[0], Sdev[1], Sdev[2]};
    double m = 0.0;
    for (int c = 0; c < 3; ++c) m += S[c] * S[c];
    m *= spec.gamma * spec.d / ((double)spec.n * spec.na);
    double f = 0.0, data = 0.0, str = 0.0, ang = 0.0, reg = 0.0, s05 = 0.0, a05 = 0.0;
    for (int q = 0; q < spec.npairs; ++q) {
        const double* t = spec.pt[q];
        f += t[OCTMC_TERM_F];
        data += t[OCTMC_TERM_DATA];
        str += t[OCTMC_TERM_STR];
        ang += t[OCTMC_TERM_ANG];
        reg += t[OCTMC_TERM_REG];
        s05 += t[OCTMC_TERM_STR05];
        a05 += t[OCTMC_TERM_ANG05];
    }
    terms[OCTMC_TERM_F] = f + m;
    terms[OCTMC_TERM_DATA] = data;
    terms[OCTMC_TERM_STR] = str;
    terms[OCTMC_TERM_ANG] = ang;
    terms[OCTMC_TERM_REG] = reg / (double)(spec.n - 1);  // every volume's R appears in n - 1 pairs
    terms[OCTMC_TERM_MEAN] = m;
    terms[OCTMC_TERM_STR05] = s05;
    terms[OCTMC_TERM_ANG05] = a05;
    terms[OCTMC_TERM_ETA] = spec.pt[0][OCTMC_TERM_ETA];  // the first pair's
    terms[OCTMC_TERM_GP] = gp;
}

int grid_n(size_t n, int cap = kMBlocks)
{
    size_t g = (n + kMB - 1) / kMB;
    if (g > (size_t)cap) g = cap;
    return g < 1 ? 1 : (int)g;
}

}  // namespace
}  // namespace octmc

using namespace octmc;

struct octmc_multi {
    octmc_ctx* ctx = nullptr;
    octmc_params params{};
    octmc_dtype dtype = OCTMC_F32;
    int n = 0, nlev = 0;
    int w[OCTMC_MAX_LEVELS] = {}, h[OCTMC_MAX_LEVELS] = {}, d[OCTMC_MAX_LEVELS] = {};
    VolumePyr vol[kMaxVol];
    std::vector<std::pair<int, int>> pairs;
    std::vector<std::unique_ptr<octmc_pair>> views;  // one per volume pair, borrowing the pyramids
    float* pdisp = nullptr;   // [npairs][2][na0][3]
    double* pgrad = nullptr;  // [npairs][2][na0][3]
    double* pterms = nullptr; // [npairs][NTERMS]
    double* sum_blk = nullptr;
    double* fsum = nullptr;  // [3] sum of all fields
    double* gp_blk = nullptr;
    std::vector<void*> owned;
    std::atomic<int> busy{0};  // a solve holds the object (taken by compare-and-swap)

    template <typename T>
    hipError_t alloc(T** p, size_t bytes)
    {
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, bytes ? bytes : 16);
        if (e == hipSuccess) {
            owned.push_back(q);
            *p = static_cast<T*>(q);
        }
        return e;
    }
    ~octmc_multi()
    {
        views.clear();
        for (void* p : owned) (void)hipFree(p);
    }
};

namespace {

// One evaluation of the n-volume objective at level `level`: ea.disp is the
// [n][na][3] field, ea.grad / ea.grad64 its gradient, ea.p a direction for
// g . p, ea.terms the terms (device), ea.pair any of the view pairs.
struct MultiEvaluator final : Evaluator {
    octmc_multi* M;
    int eval(const EvalArgs& ea, hipStream_t s) override
    {
        const int level = ea.level, np = (int)M->pairs.size();
        const size_t na = (size_t)M->w[level] * M->h[level], na0 = (size_t)M->w[0] * M->h[0];
        const size_t fb = na * 3 * sizeof(float);
        // the structural partials of all pairs in one pass that resamples every
        // volume once, where the fused kernel serves this n, storage and depth
        const bool fused = !(M->params.flags & OCTMC_MULTI_PAIRWISE) &&
                           struct_multi_supported(M->n, storage_pitch(M->d[level], M->dtype), M->dtype);
        std::vector<EvalArgs> args(np);
        for (int q = 0; q < np; ++q) {
            const float* fP = ea.disp + (size_t)M->pairs[q].first * na * 3;
            const float* fQ = ea.disp + (size_t)M->pairs[q].second * na * 3;
            args[q] = EvalArgs{M->views[q].get(), fP, M->pterms + (size_t)q * OCTMC_NTERMS, nullptr, nullptr,
                               M->pgrad + (size_t)q * 2 * na0 * 3, level, ea.eta_mode};
            args[q].skip = ea.skip;
            if (fused) {
                args[q].disp_y = fQ;  // the remaining pair kernels read the two fields where they are
                continue;
            }
            // the pair structural kernels read the two fields as one [2][na][3] array
            float* pd = M->pdisp + (size_t)q * 2 * na0 * 3;
            HIP_TRY(hipMemcpyAsync(pd, fP, fb, hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipMemcpyAsync(pd + na * 3, fQ, fb, hipMemcpyDeviceToDevice, s));
            args[q].disp = pd;
        }
        if (fused) {
            const void* vols[kMaxVol];
            float* parts[kMaxVol * (kMaxVol - 1) / 2];
            for (int V = 0; V < M->n; ++V) vols[V] = M->vol[V].s[level];
            for (int q = 0; q < np; ++q) parts[q] = M->views[q]->part;
            const Level& L = M->views[0]->lev[level];
            HIP_TRY(launch_struct_multi(vols, M->n, ea.disp, parts, L.w, L.h, L.d, L.dp, L.vol_bytes,
                                        (float)M->params.eps_huber, M->dtype, s, ea.skip));
        }
        for (int q0 = 0; q0 < np; q0 += kMaxJobs)
            OCTMC_TRY(eval_group(args.data() + q0, std::min(kMaxJobs, np - q0), s, nullptr, !fused));
        const size_t nq = (size_t)M->n * na;
        const int nsum = grid_n(nq);
        hipLaunchKernelGGL(k_field_sum, dim3(nsum), dim3(kMB), 0, s, ea.disp, nq, M->sum_blk, ea.skip);
        hipLaunchKernelGGL(k_field_sum_final, dim3(1), dim3(kMB), 0, s, M->sum_blk, nsum, M->fsum, ea.skip);
        GatherSpec gs{};
        gs.n = M->n;
        int cnt[kMaxVol] = {};
        for (int q = 0; q < np; ++q) {
            gs.pg[q] = M->pgrad + (size_t)q * 2 * na0 * 3;
            const int P = M->pairs[q].first, Q = M->pairs[q].second;
            gs.pq[P][cnt[P]] = (signed char)q;
            gs.slot[P][cnt[P]++] = 0;
            gs.pq[Q][cnt[Q]] = (signed char)q;
            gs.slot[Q][cnt[Q]++] = 1;
        }
        const octmc_params& pr = M->params;
        const double mscale = 2.0 * pr.mean_weight * M->d[level] / ((double)M->n * (double)na);
        const int ng = grid_n(na * 3);
        hipLaunchKernelGGL(k_gather, dim3(ng), dim3(kMB), 0, s, gs, na, M->fsum, mscale, ea.p, ea.grad64, ea.grad,
                           M->gp_blk, ea.skip);
        FinalSpec fs{};
        for (int q = 0; q < np; ++q) fs.pt[q] = M->pterms + (size_t)q * OCTMC_NTERMS;
        fs.npairs = np;
        fs.n = M->n;
        fs.d = M->d[level];
        fs.gamma = pr.mean_weight;
        fs.alpha = pr.alpha;
        fs.na = (double)na;
        hipLaunchKernelGGL(k_multi_final, dim3(1), dim3(64), 0, s, fs, M->fsum, M->gp_blk, ng, ea.terms, ea.skip);
        HIP_TRY(hipGetLastError());
        return OCTMC_OK;
    }
    // every launch honours ea.skip; the pair-by-pair form's field copies run
    // regardless, which is harmless: only the skipped kernels read them
    bool enqueue_only() const override { return true; }
};

// ingest one volume: staging, validity, en face image, OCTA substitution,
// pyramid
int ingest_volume(octmc_multi* M, int V, const octmc_shape* shape, const float* oct, const float* octa,
                  const float* enface, const float* valid, hipStream_t s, DevBufList& tmp)
{
    VolumePyr& P = M->vol[V];
    const int w = shape->w, h = shape->h, d = shape->d, o = P.orient;
    const int nb = o == 0 ? h : w;
    const size_t na = (size_t)w * h, nv = na * d;
    const hipMemcpyKind kind = shape->mem == OCTMC_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    float* f32 = (float*)tmp.get(nv * 4);
    if (!f32) return fail(OCTMC_E_OOM, "out of device memory (staging)");
    HIP_TRY(hipMemcpyAsync(f32, oct, nv * 4, kind, s));
    const octmc_params& pr = M->params;
    if (pr.flags & OCTMC_CHECK_NAN) {
        unsigned* ctr = (unsigned*)tmp.get(64);
        if (!ctr) return fail(OCTMC_E_OOM, "out of device memory");
        HIP_TRY(launch_fill_u32(ctr, 0u, 1, s));
        HIP_TRY(launch_count_nonfinite(f32, nv, ctr, s));
        unsigned bad = 0;
        HIP_TRY(hipMemcpyAsync(&bad, ctr, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (bad) return fail(OCTMC_E_NAN, "non-finite values in a structural volume");
    }
    // validity on the host (for the substitution table) and on the device
    std::vector<float> hv(nb, 1.0f);
    float* vd = nullptr;
    HIP_TRY(M->alloc(&vd, (size_t)nb * 4));
    if (valid) {
        HIP_TRY(hipMemcpyAsync(hv.data(), valid, (size_t)nb * 4,
                               shape->mem == OCTMC_MEM_HOST ? hipMemcpyHostToHost : hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    float* enf = nullptr;
    HIP_TRY(M->alloc(&enf, na * 4));
    if (octa) {
        HIP_TRY(M->alloc(&P.octa, nv * 4));
        HIP_TRY(hipMemcpyAsync(P.octa, octa, nv * 4, kind, s));
        if (!valid && (pr.flags & OCTMC_DETECT_INVALID)) {
            double* means = (double*)tmp.get((size_t)nb * 8);
            if (!means) return fail(OCTMC_E_OOM, "out of device memory (validity)");
            HIP_TRY(launch_validity(P.octa, w, h, d, o, means, vd, s));
            HIP_TRY(hipMemcpyAsync(hv.data(), vd, (size_t)nb * 4, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
    }
    HIP_TRY(hipMemcpyAsync(vd, hv.data(), (size_t)nb * 4, hipMemcpyHostToDevice, s));
    if (octa) {
        if (!enface && (pr.flags & OCTMC_ENFACE_PROJECT)) {
            void* scratch = tmp.get(enface_scratch_bytes(w, h, d));
            if (!scratch) return fail(OCTMC_E_OOM, "out of device memory (projection)");
            HIP_TRY(launch_enface_project(f32, P.octa, w, h, d, o, vd, nullptr, enf, nullptr, nullptr, scratch, s));
        }
        // nearest valid B-scan for the merge (the lower one on a tie)
        bool any_valid = false, any_invalid = false;
        for (int b = 0; b < nb; ++b) {
            any_valid |= hv[b] > 0.5f;
            any_invalid |= !(hv[b] > 0.5f);
        }
        if (any_valid && any_invalid) {
            std::vector<int> from(nb);
            for (int b = 0; b < nb; ++b) {
                if (hv[b] > 0.5f) {
                    from[b] = b;
                    continue;
                }
                int best = -1;
                for (int dist = 1; dist < nb && best < 0; ++dist) {
                    if (b - dist >= 0 && hv[b - dist] > 0.5f) best = b - dist;
                    else if (b + dist < nb && hv[b + dist] > 0.5f) best = b + dist;
                }
                from[b] = best;
            }
            int* dfrom = (int*)tmp.get((size_t)nb * 4);
            if (!dfrom) return fail(OCTMC_E_OOM, "out of device memory");
            HIP_TRY(hipMemcpyAsync(dfrom, from.data(), (size_t)nb * 4, hipMemcpyHostToDevice, s));
            HIP_TRY(launch_copy_bscans(P.octa, w, h, d, dfrom, o, s));
            HIP_TRY(hipStreamSynchronize(s));  // `from` is host memory
        }
        if (!enface && !(pr.flags & OCTMC_ENFACE_PROJECT)) HIP_TRY(launch_enface_mean(P.octa, (int)na, d, enf, s));
    }
    if (enface) HIP_TRY(hipMemcpyAsync(enf, enface, na * 4, kind, s));
    // pyramid
    float* cur = f32;
    float* cen = enf;
    float* cv = vd;
    for (int l = 0; l < M->nlev; ++l) {
        const int lw = M->w[l], lh = M->h[l], ld = M->d[l];
        // stored with an even pitch in 16-bit storage (odd depths padded), as a pair's levels
        const int lp = storage_pitch(ld, M->dtype);
        HIP_TRY(M->alloc(&P.s[l], (size_t)lw * lh * lp * esz(M->dtype)));
        HIP_TRY(launch_to_storage_pitched(cur, P.s[l], lw * lh, ld, lp, M->dtype, s));
        P.a[l] = cen;
        P.v[l] = cv;
        if (l + 1 < M->nlev) {
            const int w2 = M->w[l + 1], h2 = M->h[l + 1], d2 = M->d[l + 1];
            float* nxt = (float*)tmp.get((size_t)w2 * h2 * d2 * 4);
            if (!nxt) return fail(OCTMC_E_OOM, "out of device memory (pyramid)");
            HIP_TRY(launch_pyr3(cur, lw, lh, ld, nxt, s));
            float *ne = nullptr, *nvv = nullptr;
            HIP_TRY(M->alloc(&ne, (size_t)w2 * h2 * 4));
            HIP_TRY(launch_pyr2(cen, lw, lh, ne, s));
            HIP_TRY(M->alloc(&nvv, (size_t)(o == 0 ? h2 : w2) * 4));
            HIP_TRY(launch_pyr1(cv, o == 0 ? lh : lw, nvv, s));
            cur = nxt;
            cen = ne;
            cv = nvv;
        }
    }
    return OCTMC_OK;
}

int merge_multi_impl(octmc_multi* M, const float* disp, float* merged_oct, float* merged_octa, hipStream_t s)
{
    const int w = M->w[0], h = M->h[0], d = M->d[0];
    const size_t na = (size_t)w * h;
    DevBufList tmp;
    auto* grid = (unsigned long long*)tmp.get((size_t)M->n * na * 8);
    float* wo = (float*)tmp.get((size_t)M->n * na * 4);
    float* wa = (float*)tmp.get((size_t)M->n * na * 4);
    if (!grid || !wo || !wa) return fail(OCTMC_E_OOM, "out of device memory (merge)");
    HIP_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(grid), 0u, (size_t)M->n * na * 2, s));
    HIP_TRY(launch_density(disp, w, h, grid, s, M->n));
    MultiVols mv{};
    mv.n = M->n;
    for (int V = 0; V < M->n; ++V) {
        mv.vol[V] = M->vol[V].s[0];
        mv.valid[V] = merged_octa ? M->vol[V].v[0] : nullptr;
        mv.orient[V] = M->vol[V].orient;
    }
    HIP_TRY(launch_merge_weights_multi(disp, w, h, grid, mv, M->params.merge_kappa, M->params.merge_tau, wo, wa, s));
    HIP_TRY(launch_merge_volume_multi(mv, M->dtype, disp, wo, w, h, d, storage_pitch(d, M->dtype), merged_oct, s));
    if (merged_octa) {
        for (int V = 0; V < M->n; ++V) mv.vol[V] = M->vol[V].octa;
        HIP_TRY(launch_merge_volume_multi(mv, OCTMC_F32, disp, wa, w, h, d, d, merged_octa, s));
    }
    HIP_TRY(hipStreamSynchronize(s));  // the temporaries are freed on return
    return OCTMC_OK;
}

}  // namespace

extern "C" {

int octmc_multi_create(octmc_ctx* ctx, const octmc_params* params_in, const octmc_shape* shape, int32_t n,
                       const int32_t* orient, const float* const* oct, const float* const* octa,
                       const float* const* enface, const float* const* valid, void* stream, octmc_multi** out)
{
    if (!ctx || !shape || !orient || !oct || !out) return fail(OCTMC_E_INVALID, "NULL argument");
    if (n < 2 || n > kMaxVol) return fail(OCTMC_E_INVALID, "n must lie in [2, 8]");
    if (!params_in) return fail(OCTMC_E_INVALID, "params is NULL");
    const octmc_params resolved = resolve_levels(*params_in, *shape);
    const octmc_params* params = &resolved;
    OCTMC_TRY(validate_params(params));
    OCTMC_TRY(validate_shape(params, shape));
    if (params->flags & OCTMC_PREALIGN) return fail(OCTMC_E_INVALID, "OCTMC_PREALIGN is not available for n volumes");
    bool has[2] = {false, false};
    for (int V = 0; V < n; ++V) {
        if (orient[V] != 0 && orient[V] != 1) return fail(OCTMC_E_INVALID, "orientations must be 0 or 1");
        has[orient[V]] = true;
        if (!oct[V]) return fail(OCTMC_E_INVALID, "every structural volume is required");
        if (octa && !octa[V]) return fail(OCTMC_E_INVALID, "give every OCTA volume or none");
        if (enface && !enface[V]) return fail(OCTMC_E_INVALID, "give every en face image or none");
        if (valid && !valid[V]) return fail(OCTMC_E_INVALID, "give every validity vector or none");
    }
    if (!has[0] || !has[1]) return fail(OCTMC_E_INVALID, "at least one X-fast and one Y-fast scan are needed");
    if (!octa && !enface) return fail(OCTMC_E_INVALID, "need OCTA volumes or en face images");
    if ((params->flags & OCTMC_ENFACE_PROJECT) &&
        (shape->w > enface_max_bscan() || shape->h > enface_max_bscan()))
        return fail(OCTMC_E_SHAPE, "B-scans longer than 8192 A-scans for the projection");
    HIP_TRY(hipSetDevice(ctx_device(ctx)));
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto M = std::make_unique<octmc_multi>();
    M->ctx = ctx;
    M->params = *params;
    M->dtype = shape->dtype;
    M->n = n;
    M->nlev = params->levels;
    M->w[0] = shape->w;
    M->h[0] = shape->h;
    M->d[0] = shape->d;
    for (int l = 1; l < M->nlev; ++l) {
        M->w[l] = (M->w[l - 1] + 1) / 2;
        M->h[l] = (M->h[l - 1] + 1) / 2;
        M->d[l] = (M->d[l - 1] + 1) / 2;
    }
    DevBufList tmp;
    for (int V = 0; V < n; ++V) {
        M->vol[V].orient = orient[V];
        OCTMC_TRY(ingest_volume(M.get(), V, shape, oct[V], octa ? octa[V] : nullptr, enface ? enface[V] : nullptr,
                                valid ? valid[V] : nullptr, s, tmp));
    }
    // view pairs
    octmc_params pv = *params;
    pv.alpha = params->alpha / (double)(n - 1);
    pv.mean_weight = 0.0;
    const size_t na0 = (size_t)shape->w * shape->h;
    for (int P = 0; P < n; ++P)
        for (int Q = P + 1; Q < n; ++Q) {
            auto vp = std::make_unique<octmc_pair>();
            vp->ctx = ctx;
            vp->params = pv;
            vp->dtype = M->dtype;
            vp->nlev = M->nlev;
            vp->orient = M->vol[P].orient | (M->vol[Q].orient << 1);
            for (int l = 0; l < M->nlev; ++l) {
                Level& L = vp->lev[l];
                L.w = M->w[l];
                L.h = M->h[l];
                L.d = M->d[l];
                L.na = L.w * L.h;
                L.dp = storage_pitch(L.d, M->dtype);
                L.vol_bytes = (uint32_t)((size_t)L.na * L.dp * esz(M->dtype));
                L.sx = M->vol[P].s[l];
                L.sy = M->vol[Q].s[l];
                L.ax = M->vol[P].a[l];
                L.ay = M->vol[Q].a[l];
                L.vx = M->vol[P].v[l];
                L.vy = M->vol[Q].v[l];
            }
            OCTMC_TRY(pair_alloc_scratch(vp.get(), na0, s));
            M->pairs.emplace_back(P, Q);
            M->views.push_back(std::move(vp));
        }
    const size_t np = M->pairs.size();
    HIP_TRY(M->alloc(&M->pdisp, np * 2 * na0 * 3 * 4));
    HIP_TRY(M->alloc(&M->pgrad, np * 2 * na0 * 3 * 8));
    HIP_TRY(M->alloc(&M->pterms, np * OCTMC_NTERMS * 8));
    HIP_TRY(M->alloc(&M->sum_blk, (size_t)kMBlocks * 3 * 8));
    HIP_TRY(M->alloc(&M->gp_blk, (size_t)kMBlocks * 8));
    HIP_TRY(M->alloc(&M->fsum, 3 * 8));
    HIP_TRY(hipStreamSynchronize(s));  // staging is freed on return
    *out = M.release();
    return OCTMC_OK;
}

int octmc_multi_destroy(octmc_multi* m)
{
    if (m) {
        (void)hipSetDevice(ctx_device(m->ctx));
        (void)hipDeviceSynchronize();
    }
    delete m;
    return OCTMC_OK;
}

int octmc_multi_eval(octmc_multi* m, int32_t level, const float* disp, double* terms, float* grad,
                     int32_t eta_mode, void* stream)
{
    if (!m || !disp || !terms) return fail(OCTMC_E_INVALID, "multi, disp and terms are required");
    if (level < 0 || level >= m->nlev) return fail(OCTMC_E_INVALID, "level out of range");
    if (eta_mode != 0 && eta_mode != 1) return fail(OCTMC_E_INVALID, "eta_mode must be 0 or 1");
    if (m->busy.load()) return fail(OCTMC_E_BUSY, "object is in use");
    HIP_TRY(hipSetDevice(ctx_device(m->ctx)));
    MultiEvaluator ev;
    ev.M = m;
    EvalArgs ea{m->views[0].get(), disp, terms, grad, nullptr, nullptr, level, eta_mode};
    return ev.eval(ea, static_cast<hipStream_t>(stream));
}

int octmc_multi_register(octmc_multi* m, float* disp_out, float* merged_oct, float* merged_octa, octmc_report* rep,
                         void* stream)
{
    if (!m || !disp_out) return fail(OCTMC_E_INVALID, "NULL argument");
    if (merged_octa && !m->vol[0].octa) return fail(OCTMC_E_INVALID, "no OCTA volumes were given at creation");
    if (merged_octa && !merged_oct) return fail(OCTMC_E_INVALID, "merged_octa needs merged_oct");
    int idle = 0;
    if (!m->busy.compare_exchange_strong(idle, 1)) return fail(OCTMC_E_BUSY, "object is in use");
    struct Unbusy {
        octmc_multi* p;
        ~Unbusy() { p->busy.store(0); }
    } ub{m};
    HIP_TRY(hipSetDevice(ctx_device(m->ctx)));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const octmc_params& pr = m->params;
    const size_t n0 = (size_t)3 * m->n * m->w[0] * m->h[0];
    Solver sv;
    sv.m = pr.lbfgs_m;
    DevBufList mem;
    double** vecs[] = {&sv.x, &sv.g, &sv.p, &sv.xt, &sv.xprev, &sv.sc, &sv.gt, &sv.yc};
    for (double** v : vecs) {
        *v = (double*)mem.get(n0 * 8);
        if (!*v) return fail(OCTMC_E_OOM, "out of device memory (solver)");
    }
    for (int k = 0; k < sv.m; ++k) {
        sv.S[k] = (double*)mem.get(n0 * 8);
        sv.Y[k] = (double*)mem.get(n0 * 8);
        if (!sv.S[k] || !sv.Y[k]) return fail(OCTMC_E_OOM, "out of device memory (solver)");
    }
    sv.xt32 = (float*)mem.get(n0 * 4);
    if (!sv.xt32) return fail(OCTMC_E_OOM, "out of device memory (solver)");
    double *h_terms = nullptr, *h_dots = nullptr;
    HIP_TRY(hipHostMalloc(&h_terms, OCTMC_NTERMS * 8, hipHostMallocDefault));
    struct HostFree {
        double** a;
        double** b;
        ~HostFree()
        {
            if (*a) (void)hipHostFree(*a);
            if (*b) (void)hipHostFree(*b);
        }
    } hf{&h_terms, &h_dots};
    HIP_TRY(hipHostMalloc(&h_dots, (kMaxDots + 1) * 8, hipHostMallocDefault));
    if (rep) {
        std::memset(rep, 0, sizeof(*rep));
        rep->nlevels = m->nlev;
    }
    MultiEvaluator ev;
    ev.M = m;
    octmc_pair* carrier = m->views[0].get();
    for (int l = m->nlev - 1; l >= 0; --l) {
        const size_t n = (size_t)3 * m->n * m->w[l] * m->h[l];
        if (l == m->nlev - 1) {
            HIP_TRY(hipMemsetAsync(sv.x, 0, n * 8, s));
        } else {
            const size_t nc = (size_t)3 * m->n * m->w[l + 1] * m->h[l + 1];
            HIP_TRY(hipMemcpyAsync(sv.xprev, sv.x, nc * 8, hipMemcpyDeviceToDevice, s));
            HIP_TRY(launch_upsample(sv.xprev, m->w[l + 1], m->h[l + 1], sv.x, m->w[l], m->h[l], s, m->n));
        }
        sv.n = n;
        LevelRun run{carrier, l, &sv, s, n, h_terms, h_dots, &ev};
        LevelStats st;
        if (!(pr.flags & OCTMC_HOST_LINE_SEARCH) && sv.m <= kLbMaxM)
            OCTMC_TRY(run.run_device(pr, st));
        else
            OCTMC_TRY(run.run(pr, st));
        if (rep) {
            const int r = m->nlev - 1 - l;
            rep->iters[r] = st.iters;
            rep->evals[r] = st.evals;
            rep->ls_fail[r] = st.ls_fail;
            rep->f_start[r] = st.f_start;
            rep->f_end[r] = st.f_end;
            HIP_TRY(hipMemcpyAsync(h_terms, carrier->eta + l, 8, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            rep->eta[r] = h_terms[0];
        }
    }
    HIP_TRY(launch_to_f32(sv.x, disp_out, n0, s));
    if (merged_oct) OCTMC_TRY(merge_multi_impl(m, disp_out, merged_oct, merged_octa, s));
    HIP_TRY(hipStreamSynchronize(s));
    return OCTMC_OK;
}

}  // extern "C"
