// Host runtime behind the C ABI (include/octmc.h): contexts, pair ingest and
// pyramid, the evaluation sequence of the hot path, the L-BFGS level loop and
// the merge.  All vectors stay in device memory; only float64 scalars cross
// to the host (objective and directional derivative per line-search trial,
// one set of dot products per L-BFGS iteration).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "octmc_internal.h"

using namespace octmc;

namespace {
thread_local std::string g_err;
}  // namespace

int octmc::fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

namespace {

size_t esize(octmc_dtype dt) { return dt == OCTMC_F32 ? 4 : 2; }

// ---------------------------------------------------------------------------
// Scratch of octmc_eval_noalloc: one file-scope device array (each GPU the
// library runs on holds its own copy until the process ends), laid out as the
// per-A-scan partials [na][8] float32, the displacement-sum block rows
// [256][4] float64 and the combination block rows [nblk][8] float64, for at
// most kNoAllocMaxAscans A-scans.  Host code never uses the array's name as
// an address: octmc_create resolves the device address once per device
// (hipGetSymbolAddress, with that device current) and every launch takes it.
// Every kernel writes the whole part of the array it later reads, so nothing
// has to start at zero.
constexpr size_t kNoAllocPart = (size_t)OCTMC_NOALLOC_MAX_ASCANS * 8 * 4;
constexpr size_t kNoAllocSum = 256 * 4 * 8;
constexpr size_t kNoAllocComb = ((size_t)OCTMC_NOALLOC_MAX_ASCANS + 255) / 256 * 8 * 8;
constexpr size_t kNoAllocBytes = kNoAllocPart + kNoAllocSum + kNoAllocComb;
static_assert(kNoAllocPart % 256 == 0 && kNoAllocSum % 256 == 0, "sub-buffers stay 256-byte aligned");
static_assert(kNoAllocBytes == OCTMC_NOALLOC_SCRATCH_BYTES, "the size the header states");

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// The device address of `scratch` on the current device `device`, resolved
// on the first call for that device.
int scratch_address(int device, void** out)
{
    if (device < 0 || device >= kMaxDevices) return fail(OCTMC_E_INVALID, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(OCTMC_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_addr[device] = p;
    }
    *out = g_scratch_addr[device];
    return OCTMC_OK;
}

struct DevBuf {
    std::vector<void*> ptrs;
    ~DevBuf()
    {
        for (void* p : ptrs) (void)hipFree(p);
    }
};

}  // namespace

#include "runtime_types.h"

namespace {

constexpr int kSumBlocks = 256;

int nblk_combine(int na) { return (na + kRedBlock - 1) / kRedBlock; }

// ---------------------------------------------------------------------------
// hot path: one grouped evaluation over up to kMaxJobs pairs at one level

}  // namespace

int octmc::eval_group(const EvalArgs* ea, int n, hipStream_t s, hipEvent_t* ev, bool with_struct)
{
    SumJobs sj{};
    StructJobs tj{};
    CombineJobs cj{};
    sj.n = tj.n = cj.n = n;
    // one skip flag for the grouped launch (a solver enqueued ahead of its decisions)
    sj.skip = tj.skip = cj.skip = ea[0].skip;
    for (int q = 1; q < n; ++q)
        if (ea[q].skip != ea[0].skip) return fail(OCTMC_E_INVALID, "grouped evaluations must share their skip flag");
    int sb = 0, tb = 0, cb = 0;
    EvalView views[kMaxJobs];
    for (int q = 0; q < n; ++q) {
        if (ea[q].view) {
            views[q] = *ea[q].view;
        } else {
            octmc_pair* P = ea[q].pair;
            EvalView& v = views[q];
            v.L = P->lev[ea[q].level];
            v.dtype = P->dtype;
            v.params = &P->params;
            v.part = P->part;
            v.sum_blk = P->sum_blk;
            v.comb_blk = P->comb_blk;
            v.eta = P->eta + ea[q].level;
            v.orient = P->orient;
        }
    }
    const octmc_dtype dt = views[0].dtype;
    bool any_eta = false;
    for (int q = 0; q < n; ++q) {
        const EvalView& V = views[q];
        const Level& L = V.L;
        any_eta |= ea[q].eta_mode == 0;
        const octmc_params& pr = *V.params;
        if (V.dtype != dt) return fail(OCTMC_E_DTYPE, "batched pairs must share the storage type");
        const int nsum = std::min(kSumBlocks, (2 * L.na + kRedBlock - 1) / kRedBlock);
        const float* dy = ea[q].disp_y ? ea[q].disp_y : ea[q].disp + (size_t)L.na * 3;
        if (with_struct && dy != ea[q].disp + (size_t)L.na * 3)
            return fail(OCTMC_E_INVALID, "the structural kernels read both slots' fields as one [2][na][3] array");
        sj.j[q] = SumJob{{ea[q].disp, dy}, V.sum_blk, L.na, sb, nsum};
        sb += nsum;
        tj.j[q] = StructJob{L.sx, L.sy, ea[q].disp, V.part, L.w, L.h, L.d, L.na, tb, L.vol_bytes,
                            (float)pr.eps_huber, L.dp};
        tb += struct_blocks(L.w, L.h);
        const int nc = nblk_combine(L.na);
        const int blen = L.w;  // square scans: every B-scan has w A-scans
        const double f = std::floor(pr.flyback_frac * blen + 0.5);
        CombineJob c{};
        c.part = V.part;
        c.disp[0] = ea[q].disp;
        c.disp[1] = dy;
        c.grad = ea[q].grad;
        c.grad64 = ea[q].grad64;
        c.ax = L.ax;
        c.ay = L.ay;
        c.vx = L.vx;
        c.vy = L.vy;
        c.sum_blk = V.sum_blk;
        c.nsum = nsum;
        c.eta = V.eta;
        c.p = ea[q].p;
        c.blk = V.comb_blk;
        c.terms = ea[q].terms;
        c.w = L.w;
        c.h = L.h;
        c.d = L.d;
        c.na = L.na;
        c.blk_begin = cb;
        c.nblk = nc;
        c.mode = 1;
        c.orient = V.orient;
        c.delta0 = pr.delta0;
        c.eps_h = pr.eps_huber;
        c.eps_r = pr.eps_reg;
        c.alpha = pr.alpha;
        c.gamma = pr.mean_weight;
        c.wfb = 1.0 / std::sqrt(1.0 + f);
        cj.j[q] = c;
        cb += nc;
    }
    if (ev) HIP_TRY(hipEventRecord(ev[0], s));
    HIP_TRY(launch_sum(sj, sb, s));
    if (ev) HIP_TRY(hipEventRecord(ev[1], s));
    bool axial = true;
    for (int q = 0; q < n; ++q) axial &= ea[q].axial;
    if (with_struct) HIP_TRY(launch_struct(tj, (tb + 7) / 8 * 8, dt, s, axial));  // multiple of the 8 XCDs
    if (ev) HIP_TRY(hipEventRecord(ev[2], s));
    if (any_eta) {  // eta of the jobs that ask for it, before their evaluation
        CombineJobs c0{};
        c0.skip = cj.skip;
        int b0 = 0;
        for (int q = 0; q < n; ++q) {
            if (ea[q].eta_mode != 0) continue;
            CombineJob c = cj.j[q];
            c.mode = 0;
            c.grad = nullptr;
            c.grad64 = nullptr;
            c.p = nullptr;
            c.blk_begin = b0;
            b0 += c.nblk;
            c0.j[c0.n++] = c;
        }
        HIP_TRY(launch_combine(c0, b0, s));
    }
    HIP_TRY(launch_combine(cj, cb, s));
    if (ev) HIP_TRY(hipEventRecord(ev[3], s));
    return OCTMC_OK;
}

namespace {

int check_level(const octmc_pair* P, int level)
{
    if (!P) return fail(OCTMC_E_INVALID, "pair is NULL");
    if (level < 0 || level >= P->nlev) return fail(OCTMC_E_INVALID, "level out of range");
    return OCTMC_OK;
}

}  // namespace

namespace {

bool finite_param(double v) { return std::isfinite(v); }


}  // namespace

// Evaluation scratch of a pair whose finest level has na A-scans; eta = 1
// at every level.
int octmc::pair_alloc_scratch(octmc_pair* P, size_t na, hipStream_t s)
{
    HIP_TRY(P->alloc(&P->part, na * 8 * 4));
    HIP_TRY(P->alloc(&P->sum_blk, kSumBlocks * 4 * 8));
    HIP_TRY(P->alloc(&P->comb_blk, (size_t)nblk_combine((int)na) * 8 * 8));
    HIP_TRY(P->alloc(&P->eta, OCTMC_MAX_LEVELS * 8));
    HIP_TRY(P->alloc(&P->terms, OCTMC_NTERMS * 8));
    HIP_TRY(P->alloc(&P->dot_blk, (size_t)512 * (kMaxDots + 1) * 8));
    HIP_TRY(P->alloc(&P->dot_out, (kMaxDots + 1) * 8));
    HIP_TRY(P->alloc(&P->lb, sizeof(LbState)));
    static const std::vector<double> ones(OCTMC_MAX_LEVELS, 1.0);
    HIP_TRY(hipMemcpyAsync(P->eta, ones.data(), OCTMC_MAX_LEVELS * 8, hipMemcpyHostToDevice, s));
    return OCTMC_OK;
}

octmc_dtype octmc::pair_dtype(const octmc_pair* pair) { return pair->dtype; }
int octmc::pair_level_ascans(const octmc_pair* pair, int level) { return pair->lev[level].na; }
int octmc::pair_nlev(const octmc_pair* pair) { return pair->nlev; }
const octmc_params& octmc::pair_params(const octmc_pair* pair) { return pair->params; }
int octmc::pair_device(const octmc_pair* pair) { return pair->ctx->device; }
const std::vector<double>& octmc::pair_theta(const octmc_pair* pair) { return pair->theta; }

int octmc::ctx_device(const octmc_ctx* ctx) { return ctx->device; }

octmc_params octmc::resolve_levels(const octmc_params& p, const octmc_shape& shape)
{
    octmc_params r = p;
    if (p.levels != 0) return r;
    int wl = shape.w, dl = shape.d, L = 1;
    while (L < OCTMC_MAX_LEVELS && wl > kAutoCoarsest) {
        const int nw = (wl + 1) / 2, nd = (dl + 1) / 2;
        if (nw < 4 || nd < 4) break;
        wl = nw;
        dl = nd;
        ++L;
    }
    r.levels = L;
    return r;
}

int octmc::validate_params(const octmc_params* p)
{
    if (!p) return fail(OCTMC_E_INVALID, "params is NULL");
    const double vals[] = {p->alpha, p->delta0,  p->eps_huber,   p->eps_reg,  p->flyback_frac, p->mean_weight,
                           p->c1,    p->c2,      p->merge_kappa, p->merge_tau, p->gamma_tilt};
    for (double v : vals)
        if (!finite_param(v)) return fail(OCTMC_E_INVALID, "parameters must be finite");
    if (p->alpha < 0) return fail(OCTMC_E_INVALID, "alpha must be >= 0");
    if (p->delta0 < 0 || p->delta0 > 1) return fail(OCTMC_E_INVALID, "delta0 must lie in [0, 1]");
    if (!(p->eps_huber > 0) || !(p->eps_reg > 0)) return fail(OCTMC_E_INVALID, "eps_huber and eps_reg must be > 0");
    if (p->flyback_frac < 0 || p->mean_weight < 0) return fail(OCTMC_E_INVALID, "negative flyback or mean weight");
    if (p->levels < 1 || p->levels > OCTMC_MAX_LEVELS) return fail(OCTMC_E_INVALID, "levels must lie in [1, 8]");
    if (p->iters_per_level < 0) return fail(OCTMC_E_INVALID, "iters_per_level must be >= 0");
    if (p->lbfgs_m < 1 || p->lbfgs_m > 8) return fail(OCTMC_E_INVALID, "lbfgs_m must lie in [1, 8]");
    if (p->ls_max_evals < 1) return fail(OCTMC_E_INVALID, "ls_max_evals must be >= 1");
    if (!(p->c1 > 0 && p->c1 < p->c2 && p->c2 < 1)) return fail(OCTMC_E_INVALID, "need 0 < c1 < c2 < 1");
    if (p->prealign_iters < 0) return fail(OCTMC_E_INVALID, "prealign_iters must be >= 0");
    if (p->gamma_tilt < 0) return fail(OCTMC_E_INVALID, "gamma_tilt must be >= 0");
    if (p->flags & ~(OCTMC_CHECK_NAN | OCTMC_DETECT_INVALID | OCTMC_ENFACE_PROJECT | OCTMC_PREALIGN |
                     OCTMC_MULTI_PAIRWISE | OCTMC_HOST_LINE_SEARCH))
        return fail(OCTMC_E_INVALID, "unknown flags");
    return OCTMC_OK;
}

int octmc::validate_shape(const octmc_params* params, const octmc_shape* shape)
{
    if (!shape) return fail(OCTMC_E_INVALID, "shape is NULL");
    const int w = shape->w, h = shape->h, d = shape->d;
    if (shape->dtype != OCTMC_F32 && shape->dtype != OCTMC_BF16 && shape->dtype != OCTMC_F16)
        return fail(OCTMC_E_DTYPE, "unknown storage type");
    if (shape->mem != OCTMC_MEM_HOST && shape->mem != OCTMC_MEM_DEVICE)
        return fail(OCTMC_E_INVALID, "unknown memory kind");
    if (w != h) return fail(OCTMC_E_SHAPE, "only square scans (w == h) are supported");
    if (w < 4 || d < 4) return fail(OCTMC_E_SHAPE, "scans must be at least 4 x 4 x 4");
    if ((size_t)w * h * d * 4 >= (1ull << 31)) return fail(OCTMC_E_SHAPE, "volume larger than 2^31 bytes");
    int wl = w, dl = d;
    for (int l = 1; l < params->levels; ++l) {
        wl = (wl + 1) / 2;
        dl = (dl + 1) / 2;
    }
    if (wl < 4 || dl < 4) return fail(OCTMC_E_SHAPE, "too many pyramid levels for this size");
    return OCTMC_OK;
}

// Every device allocation pair_create_impl, register_impl and merge_impl make
// for one pair, each rounded up to the slab alignment.
size_t octmc::pair_footprint(const octmc_params& pr, const octmc_shape& sh, bool have_octa, bool have_valid,
                             bool merged)
{
    const size_t w = sh.w, h = sh.h, d = sh.d, na = w * h, nv = na * d;
    const size_t es = esize(sh.dtype);
    size_t t = 0;
    t += 2 * slab_bytes(nv * 4);  // float32 staging
    t += slab_bytes(64);          // counters
    t += 2 * slab_bytes(na * 4);  // en face
    if (have_octa) {
        const bool detect = !have_valid && (pr.flags & OCTMC_DETECT_INVALID);
        t += 2 * slab_bytes(nv * 4);
        if (have_valid || detect) t += slab_bytes(h * 4) + slab_bytes(w * 4);  // substitution tables
        if (detect) t += slab_bytes(h * 8) + slab_bytes(h * 4) + slab_bytes(w * 8) + slab_bytes(w * 4);
        if (pr.flags & OCTMC_ENFACE_PROJECT)
            t += slab_bytes(enface_scratch_bytes(sh.w, sh.h, sh.d)) + slab_bytes(h * 4) + slab_bytes(w * 4);
    }
    t += slab_bytes(h * 4) + slab_bytes(w * 4);  // validity
    size_t lw = w, lh = h, ld = d;
    for (int l = 0; l < pr.levels; ++l) {
        t += 2 * slab_bytes(lw * lh * (size_t)storage_pitch((int)ld, sh.dtype) * es);  // storage at its pitch
        if (l + 1 < pr.levels) {
            const size_t w2 = (lw + 1) / 2, h2 = (lh + 1) / 2, d2 = (ld + 1) / 2;
            t += 2 * slab_bytes(w2 * h2 * d2 * 4) + 2 * slab_bytes(w2 * h2 * 4) + slab_bytes(h2 * 4) +
                 slab_bytes(w2 * 4);
            lw = w2;
            lh = h2;
            ld = d2;
        }
    }
    t += slab_bytes(na * 8 * 4) + slab_bytes(kSumBlocks * 4 * 8) +
         slab_bytes((size_t)nblk_combine((int)na) * 8 * 8) + slab_bytes(OCTMC_MAX_LEVELS * 8) +
         slab_bytes(OCTMC_NTERMS * 8) + slab_bytes((size_t)512 * (kMaxDots + 1) * 8) +
         slab_bytes((kMaxDots + 1) * 8) + slab_bytes(sizeof(LbState));
    const size_t n0 = 6 * na;
    t += (size_t)(8 + 2 * pr.lbfgs_m) * slab_bytes(n0 * 8) + slab_bytes(n0 * 4);  // solver
    if (merged) t += slab_bytes(2 * na * 8) + slab_bytes(na * 16);                 // merge
    return t;
}

// ===========================================================================
// C ABI

extern "C" {

const char* octmc_version(void) { return "octmc 0.1 (gfx950)"; }

const char* octmc_last_error(void) { return g_err.c_str(); }

int octmc_params_default(octmc_params* out)
{
    if (!out) return fail(OCTMC_E_INVALID, "out is NULL");
    octmc_params p{};
    p.alpha = 1.0;
    p.delta0 = 0.5;
    p.eps_huber = 1e-3;
    p.eps_reg = 0.1;
    p.flyback_frac = 0.25;
    p.mean_weight = 1.0;
    p.levels = 0;  // automatic: the coarsest level at most kAutoCoarsest A-scans wide
    p.iters_per_level = 100;
    p.lbfgs_m = 5;
    p.ls_max_evals = 20;
    p.c1 = 1e-4;
    p.c2 = 0.9;
    p.merge_kappa = 1.0;
    p.merge_tau = 0.05;
    p.flags = 0;
    p.prealign_iters = 100;
    p.gamma_tilt = 1.0;
    *out = p;
    return OCTMC_OK;
}

int octmc_create(int device_ordinal, octmc_ctx** out)
{
    if (!out) return fail(OCTMC_E_INVALID, "out is NULL");
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device_ordinal < 0 || device_ordinal >= n) return fail(OCTMC_E_INVALID, "no such device");
    HIP_TRY(hipSetDevice(device_ordinal));
    void* scr = nullptr;
    OCTMC_TRY(scratch_address(device_ordinal, &scr));
    *out = new octmc_ctx{device_ordinal, scr};
    return OCTMC_OK;
}

int octmc_destroy(octmc_ctx* ctx)
{
    delete ctx;
    return OCTMC_OK;
}

}  // extern "C"

// Stage 1 before ingest (Fig. 1): a structural-only pair (delta0 = 0, no en
// face images) of float32 device copies of the inputs carries the stage-1
// solve; both structural volumes and the OCTA volumes are then resampled
// axially with its field, and the pair is created from the prealigned
// volumes with the remaining flags.
int octmc::prealign_create(octmc_ctx* ctx, const octmc_params* params, const octmc_shape* shape,
                           const float* oct_x, const float* oct_y, const float* octa_x, const float* octa_y,
                           const float* enface_x, const float* enface_y, const float* valid_x,
                           const float* valid_y, hipStream_t s, octmc_pair** out)
{
    const int w = shape->w, h = shape->h, d = shape->d;
    const size_t na = (size_t)w * h, nv = na * d;
    const bool host = shape->mem == OCTMC_MEM_HOST;
    const hipMemcpyKind kind = host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    const bool have_octa = octa_x && octa_y;
    DevBuf tmp;
    auto dalloc = [&](size_t bytes) -> float* {
        void* q = nullptr;
        if (hipMalloc(&q, bytes) != hipSuccess) return nullptr;
        tmp.ptrs.push_back(q);
        return static_cast<float*>(q);
    };
    const int nvol = have_octa ? 4 : 2;
    const float* src[4] = {oct_x, oct_y, octa_x, octa_y};
    float* in[4] = {nullptr, nullptr, nullptr, nullptr};
    float* pre[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int q = 0; q < nvol; ++q) {
        in[q] = dalloc(nv * 4);
        pre[q] = dalloc(nv * 4);
        if (!in[q] || !pre[q]) return fail(OCTMC_E_OOM, "out of device memory (prealignment)");
        HIP_TRY(hipMemcpyAsync(in[q], src[q], nv * 4, kind, s));
    }
    float* zero = dalloc(na * 4);
    float* dz = dalloc(2 * na * 4);
    double* th_d = (double*)dalloc(2 * (size_t)(w + h) * 8);
    if (!zero || !dz || !th_d) return fail(OCTMC_E_OOM, "out of device memory (prealignment)");
    HIP_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(zero), 0u, na, s));
    octmc_params p1 = *params;
    p1.flags &= OCTMC_CHECK_NAN | OCTMC_HOST_LINE_SEARCH;
    p1.delta0 = 0.0;  // the en face OCTA data is not used in this stage (Sec. 2.4)
    octmc_shape sh1 = *shape;
    sh1.mem = OCTMC_MEM_DEVICE;
    std::vector<double> th;
    {
        octmc_pair* P1 = nullptr;
        OCTMC_TRY(pair_create_impl(ctx, &p1, &sh1, in[0], in[1], nullptr, nullptr, zero, zero, nullptr, nullptr, s,
                                   nullptr, &P1));
        std::unique_ptr<octmc_pair> g1(P1);
        OCTMC_TRY(prealign_solve(P1, params->gamma_tilt, params->prealign_iters, th, nullptr, s));
    }
    HIP_TRY(hipMemcpyAsync(th_d, th.data(), th.size() * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_tilt_expand(th_d, w, h, nullptr, dz, s));
    for (int q = 0; q < nvol; ++q) HIP_TRY(launch_resample_z(in[q], dz + (q & 1) * na, na, d, pre[q], s));
    // en face images (depth projections, unchanged by axial shifts) and
    // validity vectors as given, on the device
    float* enf[2] = {nullptr, nullptr};
    float* val[2] = {nullptr, nullptr};
    if (enface_x && enface_y) {
        enf[0] = dalloc(na * 4);
        enf[1] = dalloc(na * 4);
        if (!enf[0] || !enf[1]) return fail(OCTMC_E_OOM, "out of device memory (prealignment)");
        HIP_TRY(hipMemcpyAsync(enf[0], enface_x, na * 4, kind, s));
        HIP_TRY(hipMemcpyAsync(enf[1], enface_y, na * 4, kind, s));
    }
    if (valid_x && valid_y) {
        val[0] = dalloc((size_t)h * 4);
        val[1] = dalloc((size_t)w * 4);
        if (!val[0] || !val[1]) return fail(OCTMC_E_OOM, "out of device memory (prealignment)");
        HIP_TRY(hipMemcpyAsync(val[0], valid_x, (size_t)h * 4, kind, s));
        HIP_TRY(hipMemcpyAsync(val[1], valid_y, (size_t)w * 4, kind, s));
    }
    octmc_params p2 = *params;
    p2.flags &= ~OCTMC_PREALIGN;
    octmc_pair* P = nullptr;
    OCTMC_TRY(pair_create_impl(ctx, &p2, &sh1, pre[0], pre[1], have_octa ? pre[2] : nullptr,
                               have_octa ? pre[3] : nullptr, enf[0], enf[1], val[0], val[1], s, nullptr, &P));
    P->theta = th;
    *out = P;
    return OCTMC_OK;
}

int octmc::pair_create_impl(octmc_ctx* ctx, const octmc_params* params, const octmc_shape* shape,
                            const float* oct_x, const float* oct_y, const float* octa_x, const float* octa_y,
                            const float* enface_x, const float* enface_y, const float* valid_x, const float* valid_y,
                            hipStream_t s, Slab* slab, octmc_pair** out)
{
    if (!ctx || !shape || !out || !oct_x || !oct_y) return fail(OCTMC_E_INVALID, "NULL argument");
    OCTMC_TRY(validate_params(params));
    OCTMC_TRY(validate_shape(params, shape));
    const int w = shape->w, h = shape->h, d = shape->d;
    const bool have_octa = octa_x && octa_y;
    const bool have_enface = enface_x && enface_y;
    const bool detect = have_octa && !valid_x && (params->flags & OCTMC_DETECT_INVALID);
    const bool project = have_octa && !have_enface && (params->flags & OCTMC_ENFACE_PROJECT);
    void* pscratch = nullptr;
    if (!have_octa && !have_enface) return fail(OCTMC_E_INVALID, "need both OCTA volumes or both en face images");
    if (project && (w > enface_max_bscan() || h > enface_max_bscan()))
        return fail(OCTMC_E_SHAPE, "B-scans longer than 8192 A-scans for the projection");
    if ((octa_x != nullptr) != (octa_y != nullptr) || (enface_x != nullptr) != (enface_y != nullptr))
        return fail(OCTMC_E_INVALID, "OCTA inputs must be given for both scans");
    if ((valid_x != nullptr) != (valid_y != nullptr)) return fail(OCTMC_E_INVALID, "give both validity vectors or none");
    HIP_TRY(hipSetDevice(ctx->device));
    if (params->flags & OCTMC_PREALIGN) {
        if (slab) return fail(OCTMC_E_INVALID, "OCTMC_PREALIGN is not available for served requests");
        return prealign_create(ctx, params, shape, oct_x, oct_y, octa_x, octa_y, enface_x, enface_y, valid_x, valid_y,
                               s, out);
    }
    auto* P = new octmc_pair();
    std::unique_ptr<octmc_pair> guard(P);
    P->slab = slab;
    P->ctx = ctx;
    P->params = *params;
    P->dtype = shape->dtype;
    P->nlev = params->levels;
    const size_t na = (size_t)w * h, nv = na * d;
    const bool host = shape->mem == OCTMC_MEM_HOST;
    const hipMemcpyKind kind = host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    DevBuf tmp;
    auto talloc = [&](size_t bytes) -> void* {
        void* q = nullptr;
        if (slab) return slab->take(bytes);  // temporaries stay in the slab until the pair is released
        if (hipMalloc(&q, bytes) != hipSuccess) return nullptr;
        tmp.ptrs.push_back(q);
        return q;
    };
    // float32 copies of the inputs
    float* f32[2] = {(float*)talloc(nv * 4), (float*)talloc(nv * 4)};
    if (!f32[0] || !f32[1]) return fail(OCTMC_E_OOM, "out of device memory (input staging)");
    HIP_TRY(hipMemcpyAsync(f32[0], oct_x, nv * 4, kind, s));
    HIP_TRY(hipMemcpyAsync(f32[1], oct_y, nv * 4, kind, s));
    std::vector<float> hvx(h, 1.0f), hvy(w, 1.0f);
    if (valid_x) {
        HIP_TRY(hipMemcpyAsync(hvx.data(), valid_x, h * 4, host ? hipMemcpyHostToHost : hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(hvy.data(), valid_y, w * 4, host ? hipMemcpyHostToHost : hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    unsigned* ctr = nullptr;
    HIP_TRY(P->alloc(&ctr, 64));
    HIP_TRY(launch_fill_u32(ctr, 0u, 16, s));
    P->counters = ctr;
    if (params->flags & OCTMC_CHECK_NAN) {
        HIP_TRY(launch_count_nonfinite(f32[0], nv, ctr + 8, s));
        HIP_TRY(launch_count_nonfinite(f32[1], nv, ctr + 8, s));
        unsigned bad = 0;
        HIP_TRY(hipMemcpyAsync(&bad, ctr + 8, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (bad) return fail(OCTMC_E_NAN, "non-finite values in the structural volumes");
    }
    // OCTA volumes: keep for the merge, replace invalid B-scans by their
    // nearest valid neighbour (Sec. 2.3, 2.5), then project
    float* enf[2] = {nullptr, nullptr};
    HIP_TRY(P->alloc(&enf[0], na * 4));
    HIP_TRY(P->alloc(&enf[1], na * 4));
    if (have_octa) {
        const float* src[2] = {octa_x, octa_y};
        for (int V = 0; V < 2; ++V) {
            HIP_TRY(P->alloc(&P->octa[V], nv * 4));
            HIP_TRY(hipMemcpyAsync(P->octa[V], src[V], nv * 4, kind, s));
            if (detect) {  // B-scan validity from the OCTA volume (Sec. 2.2)
                std::vector<float>& hv = V == 0 ? hvx : hvy;
                double* means = (double*)talloc(hv.size() * 8);
                float* dv = (float*)talloc(hv.size() * 4);
                if (!means || !dv) return fail(OCTMC_E_OOM, "out of device memory (validity)");
                HIP_TRY(launch_validity(P->octa[V], w, h, d, V, means, dv, s));
                HIP_TRY(hipMemcpyAsync(hv.data(), dv, hv.size() * 4, hipMemcpyDeviceToHost, s));
                HIP_TRY(hipStreamSynchronize(s));
            }
            const std::vector<float>& val = V == 0 ? hvx : hvy;
            const int nb = V == 0 ? h : w;
            if (project) {  // Sec. 2.3, from the OCTA volume before substitution
                if (!pscratch) pscratch = talloc(enface_scratch_bytes(w, h, d));
                float* dv = (float*)talloc((size_t)nb * 4);
                if (!pscratch || !dv) return fail(OCTMC_E_OOM, "out of device memory (projection)");
                HIP_TRY(hipMemcpyAsync(dv, val.data(), (size_t)nb * 4, hipMemcpyHostToDevice, s));
                HIP_TRY(launch_enface_project(f32[V], P->octa[V], w, h, d, V, dv, nullptr, enf[V], nullptr, nullptr,
                                              pscratch, s));
                HIP_TRY(hipStreamSynchronize(s));  // `val` is host memory
            }
            std::vector<int> from(nb);
            bool any_valid = false, any_invalid = false;
            for (int b = 0; b < nb; ++b) {
                any_valid |= val[b] > 0.5f;
                any_invalid |= !(val[b] > 0.5f);
            }
            if (any_valid && any_invalid) {
                for (int b = 0; b < nb; ++b) {
                    if (val[b] > 0.5f) {
                        from[b] = b;
                        continue;
                    }
                    int best = -1;
                    for (int dist = 1; dist < nb && best < 0; ++dist) {
                        if (b - dist >= 0 && val[b - dist] > 0.5f) best = b - dist;
                        else if (b + dist < nb && val[b + dist] > 0.5f) best = b + dist;
                    }
                    from[b] = best;
                }
                int* dfrom = (int*)talloc(nb * 4);
                if (!dfrom) return fail(OCTMC_E_OOM, "out of device memory");
                HIP_TRY(hipMemcpyAsync(dfrom, from.data(), nb * 4, hipMemcpyHostToDevice, s));
                HIP_TRY(launch_copy_bscans(P->octa[V], w, h, d, dfrom, V, s));
                HIP_TRY(hipStreamSynchronize(s));  // `from` is host memory
            }
            if (!have_enface && !project) HIP_TRY(launch_enface_mean(P->octa[V], (int)na, d, enf[V], s));
        }
    }
    if (have_enface) {
        HIP_TRY(hipMemcpyAsync(enf[0], enface_x, na * 4, kind, s));
        HIP_TRY(hipMemcpyAsync(enf[1], enface_y, na * 4, kind, s));
    }
    // pyramid: float32 at every level, stored in the storage type
    float* cur[2] = {f32[0], f32[1]};
    float* cen[2] = {enf[0], enf[1]};
    float *cvx = nullptr, *cvy = nullptr;
    HIP_TRY(P->alloc(&cvx, h * 4));
    HIP_TRY(P->alloc(&cvy, w * 4));
    HIP_TRY(hipMemcpyAsync(cvx, hvx.data(), h * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(cvy, hvy.data(), w * 4, hipMemcpyHostToDevice, s));
    int lw = w, lh = h, ld = d;
    for (int l = 0; l < P->nlev; ++l) {
        Level& L = P->lev[l];
        L.w = lw;
        L.h = lh;
        L.d = ld;
        L.na = lw * lh;
        // 16-bit storage of an odd depth gets one padding sample per A-scan, so
        // that the two-samples-per-lane structural kernel serves every level
        L.dp = storage_pitch(ld, P->dtype);
        const size_t lnv = (size_t)L.na * L.dp;
        L.vol_bytes = (uint32_t)(lnv * esize(P->dtype));
        void* st[2];
        for (int V = 0; V < 2; ++V) {
            HIP_TRY(P->alloc(&st[V], lnv * esize(P->dtype)));
            HIP_TRY(launch_to_storage_pitched(cur[V], st[V], L.na, ld, L.dp, P->dtype, s));
        }
        L.sx = st[0];
        L.sy = st[1];
        L.ax = cen[0];
        L.ay = cen[1];
        L.vx = cvx;
        L.vy = cvy;
        if (l + 1 < P->nlev) {
            const int w2 = (lw + 1) / 2, h2 = (lh + 1) / 2, d2 = (ld + 1) / 2;
            float* nxt[2];
            for (int V = 0; V < 2; ++V) {
                nxt[V] = (float*)talloc((size_t)w2 * h2 * d2 * 4);
                if (!nxt[V]) return fail(OCTMC_E_OOM, "out of device memory (pyramid)");
                HIP_TRY(launch_pyr3(cur[V], lw, lh, ld, nxt[V], s));
            }
            float* ne[2];
            for (int V = 0; V < 2; ++V) {
                HIP_TRY(P->alloc(&ne[V], (size_t)w2 * h2 * 4));
                HIP_TRY(launch_pyr2(cen[V], lw, lh, ne[V], s));
            }
            float *nvx, *nvy;
            HIP_TRY(P->alloc(&nvx, h2 * 4));
            HIP_TRY(P->alloc(&nvy, w2 * 4));
            HIP_TRY(launch_pyr1(cvx, lh, nvx, s));
            HIP_TRY(launch_pyr1(cvy, lw, nvy, s));
            cur[0] = nxt[0];
            cur[1] = nxt[1];
            cen[0] = ne[0];
            cen[1] = ne[1];
            cvx = nvx;
            cvy = nvy;
            lw = w2;
            lh = h2;
            ld = d2;
        }
    }
    OCTMC_TRY(pair_alloc_scratch(P, na, s));
    HIP_TRY(hipStreamSynchronize(s));  // temporaries are freed on return
    *out = guard.release();
    return OCTMC_OK;
}

extern "C" {

int octmc_pair_create(octmc_ctx* ctx, const octmc_params* params, const octmc_shape* shape, const float* oct_x,
                      const float* oct_y, const float* octa_x, const float* octa_y, const float* enface_x,
                      const float* enface_y, const float* valid_x, const float* valid_y, void* stream,
                      octmc_pair** out)
{
    octmc_params pr{};
    if (params && shape) pr = resolve_levels(*params, *shape);
    return pair_create_impl(ctx, params && shape ? &pr : params, shape, oct_x, oct_y, octa_x, octa_y, enface_x,
                            enface_y, valid_x, valid_y, static_cast<hipStream_t>(stream), nullptr, out);
}

int octmc_validity_from_octa(octmc_ctx* ctx, const octmc_shape* shape, const float* octa, int32_t scan,
                             float* valid_out, void* stream)
{
    if (!ctx || !shape || !octa || !valid_out) return fail(OCTMC_E_INVALID, "NULL argument");
    if (scan != 0 && scan != 1) return fail(OCTMC_E_INVALID, "scan must be 0 (X-fast) or 1 (Y-fast)");
    if (shape->mem != OCTMC_MEM_HOST && shape->mem != OCTMC_MEM_DEVICE)
        return fail(OCTMC_E_INVALID, "unknown memory kind");
    const int w = shape->w, h = shape->h, d = shape->d;
    if (w < 1 || h < 1 || d < 1) return fail(OCTMC_E_SHAPE, "empty volume");
    const size_t nv = (size_t)w * h * d;
    if (nv * 4 >= (1ull << 31)) return fail(OCTMC_E_SHAPE, "volume larger than 2^31 bytes");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    DevBuf tmp;
    const float* vol = octa;
    if (shape->mem == OCTMC_MEM_HOST) {
        void* q = nullptr;
        HIP_TRY(hipMalloc(&q, nv * 4));
        tmp.ptrs.push_back(q);
        HIP_TRY(hipMemcpyAsync(q, octa, nv * 4, hipMemcpyHostToDevice, s));
        vol = static_cast<const float*>(q);
    }
    void* means = nullptr;
    HIP_TRY(hipMalloc(&means, (size_t)(scan == 0 ? h : w) * 8));
    tmp.ptrs.push_back(means);
    HIP_TRY(launch_validity(vol, w, h, d, scan, static_cast<double*>(means), valid_out, s));
    HIP_TRY(hipStreamSynchronize(s));  // the temporaries are freed on return
    return OCTMC_OK;
}

int octmc_enface_workspace_size(int32_t w, int32_t h, int32_t d, uint64_t* bytes)
{
    if (!bytes) return fail(OCTMC_E_INVALID, "NULL argument");
    if (w < 1 || h < 1 || d < 1) return fail(OCTMC_E_SHAPE, "empty volume");
    *bytes = enface_scratch_bytes(w, h, d);
    return OCTMC_OK;
}

int octmc_enface_project(octmc_ctx* ctx, const octmc_shape* shape, const float* oct, const float* octa,
                         int32_t scan, const float* valid, const double* fixed, float* enface_out,
                         int32_t* count_out, double* stats_out, void* workspace, uint64_t workspace_bytes,
                         void* stream)
{
    if (!ctx || !shape || !oct || !octa || !enface_out) return fail(OCTMC_E_INVALID, "NULL argument");
    if (scan != 0 && scan != 1) return fail(OCTMC_E_INVALID, "scan must be 0 (X-fast) or 1 (Y-fast)");
    if (shape->mem != OCTMC_MEM_HOST && shape->mem != OCTMC_MEM_DEVICE)
        return fail(OCTMC_E_INVALID, "unknown memory kind");
    const int w = shape->w, h = shape->h, d = shape->d;
    if (w < 1 || h < 1 || d < 1) return fail(OCTMC_E_SHAPE, "empty volume");
    if (w > enface_max_bscan() || h > enface_max_bscan()) return fail(OCTMC_E_SHAPE, "B-scans longer than 8192 A-scans");
    const size_t nv = (size_t)w * h * d, nb = scan == 0 ? h : w;
    if (nv * 4 >= (1ull << 31)) return fail(OCTMC_E_SHAPE, "volume larger than 2^31 bytes");
    if (fixed && !(fixed[0] == fixed[0] && fixed[1] == fixed[1])) return fail(OCTMC_E_INVALID, "fixed mapping is NaN");
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    DevBuf tmp;
    auto dalloc = [&](size_t bytes) -> void* {
        void* q = nullptr;
        if (hipMalloc(&q, bytes) != hipSuccess) return nullptr;
        tmp.ptrs.push_back(q);
        return q;
    };
    if (workspace && workspace_bytes < enface_scratch_bytes(w, h, d))
        return fail(OCTMC_E_INVALID, "workspace smaller than octmc_enface_workspace_size");
    void* scratch = workspace ? workspace : dalloc(enface_scratch_bytes(w, h, d));
    if (!scratch) return fail(OCTMC_E_OOM, "out of device memory (projection scratch)");
    const float *o = oct, *a = octa, *v = valid;
    if (shape->mem == OCTMC_MEM_HOST) {
        float* q = (float*)dalloc(2 * nv * 4 + nb * 4);
        if (!q) return fail(OCTMC_E_OOM, "out of device memory (input copies)");
        HIP_TRY(hipMemcpyAsync(q, oct, nv * 4, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(q + nv, octa, nv * 4, hipMemcpyHostToDevice, s));
        o = q;
        a = q + nv;
        if (valid) {
            HIP_TRY(hipMemcpyAsync(q + 2 * nv, valid, nb * 4, hipMemcpyHostToDevice, s));
            v = q + 2 * nv;
        }
    }
    HIP_TRY(launch_enface_project(o, a, w, h, d, scan, v, fixed, enface_out, count_out, stats_out, scratch, s));
    if (!tmp.ptrs.empty() || stats_out) HIP_TRY(hipStreamSynchronize(s));  // temporaries are freed on return
    return OCTMC_OK;
}

int octmc_pair_destroy(octmc_pair* pair)
{
    if (pair && !pair->slab) {  // a slab's owner orders its release after the pair's work
        (void)hipSetDevice(pair->ctx->device);
        (void)hipDeviceSynchronize();
    }
    delete pair;
    return OCTMC_OK;
}

int octmc_pair_levels(const octmc_pair* pair, int32_t* levels)
{
    if (!pair || !levels) return fail(OCTMC_E_INVALID, "NULL argument");
    *levels = pair->nlev;
    return OCTMC_OK;
}

int octmc_pair_level_shape(const octmc_pair* pair, int32_t level, int32_t* w, int32_t* h, int32_t* d)
{
    OCTMC_TRY(check_level(pair, level));
    if (w) *w = pair->lev[level].w;
    if (h) *h = pair->lev[level].h;
    if (d) *d = pair->lev[level].d;
    return OCTMC_OK;
}

int octmc_eval(octmc_pair* pair, int32_t level, const float* disp, double* terms, float* grad, int32_t eta_mode,
               void* stream)
{
    OCTMC_TRY(check_level(pair, level));
    if (!disp || !terms) return fail(OCTMC_E_INVALID, "disp and terms are required");
    if (eta_mode != 0 && eta_mode != 1) return fail(OCTMC_E_INVALID, "eta_mode must be 0 or 1");
    HIP_TRY(hipSetDevice(pair->ctx->device));
    EvalArgs ea{pair, disp, terms, grad, nullptr, nullptr, level, eta_mode};
    return eval_group(&ea, 1, static_cast<hipStream_t>(stream));
}

int octmc_eval_noalloc(octmc_ctx* ctx, const octmc_params* params, const octmc_shape* shape, const void* sx,
                       const void* sy, const float* ax, const float* ay, const float* vx, const float* vy,
                       const float* disp, double* eta, double* terms, float* grad, int32_t eta_mode, void* stream)
{
    if (!ctx || !params || !shape) return fail(OCTMC_E_INVALID, "ctx, params and shape are required");
    if (!sx || !sy || !ax || !ay || !vx || !vy || !disp || !eta || !terms)
        return fail(OCTMC_E_INVALID, "volumes, en face images, validity, disp, eta and terms are required");
    if (eta_mode != 0 && eta_mode != 1) return fail(OCTMC_E_INVALID, "eta_mode must be 0 or 1");
    octmc_params pr = *params;
    pr.levels = 1;  // one level: the pyramid depth plays no part here
    OCTMC_TRY(validate_params(&pr));
    if (shape->mem != OCTMC_MEM_DEVICE) return fail(OCTMC_E_INVALID, "octmc_eval_noalloc takes device inputs");
    OCTMC_TRY(validate_shape(&pr, shape));
    const int w = shape->w, h = shape->h, d = shape->d;
    const size_t na = (size_t)w * h;
    if (na > (size_t)OCTMC_NOALLOC_MAX_ASCANS)
        return fail(OCTMC_E_SHAPE, "w * h exceeds OCTMC_NOALLOC_MAX_ASCANS (the static scratch of octmc_eval_noalloc)");
    if (!ctx->noalloc_scratch) return fail(OCTMC_E_DEVICE, "the context holds no scratch address");
    HIP_TRY(hipSetDevice(ctx->device));
    EvalView v;
    v.L.w = w;
    v.L.h = h;
    v.L.d = d;
    v.L.na = (int)na;
    v.L.dp = d;  // the caller's volumes: [h][w][d]
    v.L.sx = const_cast<void*>(sx);  // read only
    v.L.sy = const_cast<void*>(sy);
    v.L.ax = const_cast<float*>(ax);
    v.L.ay = const_cast<float*>(ay);
    v.L.vx = const_cast<float*>(vx);
    v.L.vy = const_cast<float*>(vy);
    v.L.vol_bytes = (uint32_t)(na * d * esize(shape->dtype));
    v.dtype = shape->dtype;
    v.params = &pr;
    char* base = static_cast<char*>(ctx->noalloc_scratch);
    v.part = reinterpret_cast<float*>(base);
    v.sum_blk = reinterpret_cast<double*>(base + kNoAllocPart);
    v.comb_blk = reinterpret_cast<double*>(base + kNoAllocPart + kNoAllocSum);
    v.eta = eta;
    v.orient = 2;
    EvalArgs ea{nullptr, disp, terms, grad, nullptr, nullptr, 0, eta_mode};
    ea.view = &v;
    return eval_group(&ea, 1, static_cast<hipStream_t>(stream));
}

int octmc_eval_profile(octmc_pair* pair, int32_t level, const float* disp, double* terms, float* grad,
                       int32_t eta_mode, float* stage_ms, void* stream)
{
    OCTMC_TRY(check_level(pair, level));
    if (!disp || !terms || !stage_ms) return fail(OCTMC_E_INVALID, "disp, terms and stage_ms are required");
    if (eta_mode != 0 && eta_mode != 1) return fail(OCTMC_E_INVALID, "eta_mode must be 0 or 1");
    HIP_TRY(hipSetDevice(pair->ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t ev[4] = {};
    for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
    struct Ev {
        hipEvent_t* e;
        ~Ev()
        {
            for (int k = 0; k < 4; ++k) (void)hipEventDestroy(e[k]);
        }
    } guard{ev};
    EvalArgs ea{pair, disp, terms, grad, nullptr, nullptr, level, eta_mode};
    OCTMC_TRY(eval_group(&ea, 1, s, ev));
    HIP_TRY(hipEventSynchronize(ev[3]));
    for (int k = 0; k < 3; ++k) HIP_TRY(hipEventElapsedTime(stage_ms + k, ev[k], ev[k + 1]));
    return OCTMC_OK;
}

int octmc_eval_batched(octmc_pair* const* pairs, int32_t npairs, int32_t level, const float* disp, double* terms,
                       float* grad, int32_t eta_mode, void* stream)
{
    if (!pairs || npairs < 1 || !disp || !terms) return fail(OCTMC_E_INVALID, "bad batched arguments");
    if (eta_mode != 0 && eta_mode != 1) return fail(OCTMC_E_INVALID, "eta_mode must be 0 or 1");
    for (int q = 0; q < npairs; ++q) {
        OCTMC_TRY(check_level(pairs[q], level));
        for (int r = 0; r < q; ++r)
            if (pairs[r] == pairs[q]) return fail(OCTMC_E_INVALID, "a pair appears twice in the batch");
    }
    const Level& L0 = pairs[0]->lev[level];
    for (int q = 1; q < npairs; ++q) {
        const Level& L = pairs[q]->lev[level];
        if (L.w != L0.w || L.h != L0.h || L.d != L0.d) return fail(OCTMC_E_SHAPE, "batched pairs differ in shape");
    }
    HIP_TRY(hipSetDevice(pairs[0]->ctx->device));
    const size_t nd = (size_t)2 * L0.na * 3;
    for (int q0 = 0; q0 < npairs; q0 += kMaxJobs) {
        const int cnt = std::min(kMaxJobs, npairs - q0);
        EvalArgs ea[kMaxJobs];
        for (int q = 0; q < cnt; ++q)
            ea[q] = EvalArgs{pairs[q0 + q], disp + (q0 + q) * nd, terms + (size_t)(q0 + q) * OCTMC_NTERMS,
                             grad ? grad + (q0 + q) * nd : nullptr, nullptr, nullptr, level, eta_mode};
        OCTMC_TRY(eval_group(ea, cnt, static_cast<hipStream_t>(stream)));
    }
    return OCTMC_OK;
}

}  // extern "C"

int octmc::merge_impl(octmc_pair* pair, const float* disp, float* merged_oct, float* merged_octa, hipStream_t s,
                      Slab* slab)
{
    if (!pair || !disp || !merged_oct) return fail(OCTMC_E_INVALID, "NULL argument");
    if (merged_octa && !pair->octa[0]) return fail(OCTMC_E_INVALID, "no OCTA volumes were given at creation");
    HIP_TRY(hipSetDevice(pair->ctx->device));
    const Level& L = pair->lev[0];
    DevBuf tmp;
    unsigned long long* grid = nullptr;
    float4* wts = nullptr;
    if (slab) {
        grid = static_cast<unsigned long long*>(slab->take((size_t)2 * L.na * 8));
        wts = static_cast<float4*>(slab->take((size_t)L.na * 16));
        if (!grid || !wts) return fail(OCTMC_E_OOM, "slab exhausted (merge)");
    } else {
        HIP_TRY(hipMalloc(&grid, (size_t)2 * L.na * 8));
        tmp.ptrs.push_back(grid);
        HIP_TRY(hipMalloc(&wts, (size_t)L.na * 16));
        tmp.ptrs.push_back(wts);
    }
    HIP_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(grid), 0u, (size_t)4 * L.na, s));
    HIP_TRY(launch_density(disp, L.w, L.h, grid, s));
    HIP_TRY(launch_merge_weights(disp, L.w, L.h, grid, merged_octa ? L.vx : nullptr, merged_octa ? L.vy : nullptr,
                                 pair->params.merge_kappa, pair->params.merge_tau, wts, s));
    HIP_TRY(launch_merge_volume(L.sx, L.sy, pair->dtype, disp, wts, 0, L.w, L.h, L.d, L.dp, merged_oct, s));
    if (merged_octa)
        HIP_TRY(launch_merge_volume(pair->octa[0], pair->octa[1], OCTMC_F32, disp, wts, 1, L.w, L.h, L.d, L.d,
                                    merged_octa, s));
    HIP_TRY(hipStreamSynchronize(s));
    return OCTMC_OK;
}

int octmc::register_impl(octmc_pair* pair, float* disp_out, float* merged_oct, float* merged_octa, octmc_report* rep,
                         hipStream_t s, Evaluator* ev, Slab* slab, double* h_terms_in, double* h_dots_in)
{
    if (!pair || !disp_out) return fail(OCTMC_E_INVALID, "NULL argument");
    if (merged_octa && !pair->octa[0]) return fail(OCTMC_E_INVALID, "no OCTA volumes were given at creation");
    int idle = 0;
    if (!pair->busy.compare_exchange_strong(idle, 1)) return fail(OCTMC_E_BUSY, "pair is in use");
    struct Unbusy {
        octmc_pair* p;
        ~Unbusy() { p->busy.store(0); }
    } ub{pair};
    HIP_TRY(hipSetDevice(pair->ctx->device));
    DirectEvaluator direct;
    if (!ev) ev = &direct;
    const octmc_params& pr = pair->params;
    const size_t n0 = (size_t)6 * pair->lev[0].na;
    Solver sv;
    sv.m = pr.lbfgs_m;
    DevBuf mem;
    auto dalloc = [&](double** p) -> int {
        if (slab) {
            *p = static_cast<double*>(slab->take(n0 * 8));
            if (!*p) return fail(OCTMC_E_OOM, "slab exhausted (solver)");
            return OCTMC_OK;
        }
        HIP_TRY(hipMalloc(p, n0 * 8));
        mem.ptrs.push_back(*p);
        return OCTMC_OK;
    };
    OCTMC_TRY(dalloc(&sv.x));
    OCTMC_TRY(dalloc(&sv.g));
    OCTMC_TRY(dalloc(&sv.p));
    OCTMC_TRY(dalloc(&sv.xt));
    OCTMC_TRY(dalloc(&sv.xprev));
    OCTMC_TRY(dalloc(&sv.sc));
    OCTMC_TRY(dalloc(&sv.gt));
    OCTMC_TRY(dalloc(&sv.yc));
    for (int k = 0; k < sv.m; ++k) {
        OCTMC_TRY(dalloc(&sv.S[k]));
        OCTMC_TRY(dalloc(&sv.Y[k]));
    }
    if (slab) {
        sv.xt32 = static_cast<float*>(slab->take(n0 * 4));
        if (!sv.xt32) return fail(OCTMC_E_OOM, "slab exhausted (solver)");
    } else {
        HIP_TRY(hipMalloc(&sv.xt32, n0 * 4));
        mem.ptrs.push_back(sv.xt32);
    }
    double *h_terms = h_terms_in, *h_dots = h_dots_in;
    struct HostFree {
        double *a = nullptr, *b = nullptr;
        ~HostFree()
        {
            if (a) (void)hipHostFree(a);
            if (b) (void)hipHostFree(b);
        }
    } hf;
    if (!h_terms) {
        HIP_TRY(hipHostMalloc(&h_terms, OCTMC_NTERMS * 8, hipHostMallocDefault));
        hf.a = h_terms;
    }
    if (!h_dots) {
        HIP_TRY(hipHostMalloc(&h_dots, (kMaxDots + 1) * 8, hipHostMallocDefault));
        hf.b = h_dots;
    }
    if (rep) {
        std::memset(rep, 0, sizeof(*rep));
        rep->nlevels = pair->nlev;
    }
    // the iteration's decisions on the device when the evaluator only
    // enqueues work and the history fits one keyed dot-product pass
    const bool device_ls = ev->enqueue_only() && !(pr.flags & OCTMC_HOST_LINE_SEARCH) && sv.m <= kLbMaxM;
    for (int l = pair->nlev - 1; l >= 0; --l) {
        const Level& L = pair->lev[l];
        const size_t n = (size_t)6 * L.na;
        if (l == pair->nlev - 1) {
            HIP_TRY(hipMemsetAsync(sv.x, 0, n * 8, s));
        } else {
            const Level& C = pair->lev[l + 1];
            HIP_TRY(hipMemcpyAsync(sv.xprev, sv.x, (size_t)6 * C.na * 8, hipMemcpyDeviceToDevice, s));
            HIP_TRY(launch_upsample(sv.xprev, C.w, C.h, sv.x, L.w, L.h, s));
        }
        sv.n = n;
        LevelRun run{pair, l, &sv, s, n, h_terms, h_dots, ev};
        LevelStats st;
        if (device_ls)
            OCTMC_TRY(run.run_device(pr, st));
        else
            OCTMC_TRY(run.run(pr, st));
        if (rep) {
            const int r = pair->nlev - 1 - l;
            rep->iters[r] = st.iters;
            rep->evals[r] = st.evals;
            rep->ls_fail[r] = st.ls_fail;
            rep->f_start[r] = st.f_start;
            rep->f_end[r] = st.f_end;
            HIP_TRY(hipMemcpyAsync(h_terms, pair->eta + l, 8, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            rep->eta[r] = h_terms[0];
        }
    }
    HIP_TRY(launch_to_f32(sv.x, disp_out, n0, s));
    if (merged_oct) OCTMC_TRY(merge_impl(pair, disp_out, merged_oct, merged_octa, s, slab));
    HIP_TRY(hipStreamSynchronize(s));
    return OCTMC_OK;
}

extern "C" {

int octmc_merge(octmc_pair* pair, const float* disp, float* merged_oct, float* merged_octa, void* stream)
{
    return merge_impl(pair, disp, merged_oct, merged_octa, static_cast<hipStream_t>(stream), nullptr);
}

int octmc_register(octmc_pair* pair, float* disp_out, float* merged_oct, float* merged_octa, octmc_report* rep,
                   void* stream)
{
    return register_impl(pair, disp_out, merged_oct, merged_octa, rep, static_cast<hipStream_t>(stream), nullptr,
                         nullptr, nullptr, nullptr);
}

}  // extern "C"
