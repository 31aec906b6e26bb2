// Stage 1, rough axial prealignment (Fig. 1, Sec. 2.1 "optimization"): the
// objective of Eq. 1 restricted to axial displacements with one offset and
// one tilt per B-scan, plus the tilt normalisation T, minimised by L-BFGS on
// the factor-2 pyramid; and the axial resampling that turns its result into
// the prealigned volumes.
//
// The stage evaluates the pair's objective with the library's kernels at the
// field expanded from theta (kernels_prealign.hip), reduces the field
// gradient back onto theta and adds T on the device.  theta has 2 (h + w)
// values at a level of w x h A-scans; it is solved by the same L-BFGS
// iteration as the 3-D registration (LevelRun), with its decisions on the
// device unless OCTMC_HOST_LINE_SEARCH asks for the host form.
//
// T is defined only in earlier work that is not available.  Reading: a
// quadratic penalty on the sum of each scan's tilts,
//   T = sum_V gamma_t d n_f (n_f^2 - 1) / (24 n_b) (sum_b t_b)^2,
// which fixes the two degrees of freedom the data term cannot see (a common
// plane a x + b y added to both scans' fields) as M fixes the translations;
// a uniform tilt tau then costs gamma_t d N_A var_f tau^2 / 2.
#include <cmath>
#include <vector>

#include "runtime_types.h"

namespace octmc {
namespace {

struct DevMem {
    std::vector<void*> p;
    ~DevMem()
    {
        for (void* q : p) (void)hipFree(q);
    }
    template <typename T>
    T* get(size_t n)
    {
        void* q = nullptr;
        if (hipMalloc(&q, n * sizeof(T) ? n * sizeof(T) : 16) != hipSuccess) return nullptr;
        p.push_back(q);
        return static_cast<T*>(q);
    }
};

// Level transition: the fine field is twice the coarse field at the coarse
// position ((f - 0.5)/2, (b - 0.5)/2), linear along the fast axis as the
// field is, interpolated linearly between B-scans and clamped to the first
// and last: t = t_c(u), z = 2 z_c(u) + t (n_f - 2 n_fc) / 2, u = (b - 0.5)/2.
std::vector<double> upsample_theta(const std::vector<double>& c, int wc, int hc, int wf, int hf)
{
    std::vector<double> f(2 * (size_t)(wf + hf), 0.0);
    for (int V = 0; V < 2; ++V) {
        const int nbc = V == 0 ? hc : wc, nfc = V == 0 ? wc : hc;
        const int nbf = V == 0 ? hf : wf, nff = V == 0 ? wf : hf;
        const size_t offc = V == 0 ? 0 : 2 * (size_t)hc, offf = V == 0 ? 0 : 2 * (size_t)hf;
        for (int b = 0; b < nbf; ++b) {
            double u = std::min(std::max((b - 0.5) / 2.0, 0.0), (double)(nbc - 1));
            const int b0 = (int)std::floor(u), b1 = std::min(b0 + 1, nbc - 1);
            const double fr = u - b0;
            const double z = (1.0 - fr) * c[offc + 2 * b0] + fr * c[offc + 2 * b1];
            const double t = (1.0 - fr) * c[offc + 2 * b0 + 1] + fr * c[offc + 2 * b1 + 1];
            f[offf + 2 * b + 1] = t;
            f[offf + 2 * b] = 2.0 * z + t * 0.5 * (nff - 2.0 * nfc);
        }
    }
    return f;
}

// One stage-1 evaluation at one level, as an evaluator of the L-BFGS
// iteration: theta is ea.x64 (float64, device), its gradient goes to
// ea.grad64 and the terms, with F + T and g . p, to ea.terms.  The field and
// its gradient live in device buffers sized for the finest level.  Every
// launch honours ea.skip, so the device form of the iteration can enqueue it
// ahead of its decisions.
struct StageEvaluator final : Evaluator {
    octmc_pair* P;
    int w, h, d;
    double gamma;
    double* terms_d;  // the field objective's terms (without T)
    double* T_d;      // T of the last evaluation
    float* disp;
    float* grad;
    StageEvaluator(octmc_pair* p, int w_, int h_, int d_, double g, double* terms, double* T, float* di, float* gr)
        : P(p), w(w_), h(h_), d(d_), gamma(g), terms_d(terms), T_d(T), disp(di), grad(gr)
    {
    }
    int eval(const EvalArgs& ea, hipStream_t s) override
    {
        HIP_TRY(launch_tilt_expand(ea.x64, w, h, disp, nullptr, s, ea.skip));
        EvalArgs e{P, disp, terms_d, grad, nullptr, nullptr, ea.level, 1};
        e.axial = true;  // the field has dx = dy = 0; only its z gradient is used
        e.skip = ea.skip;
        OCTMC_TRY(eval_group(&e, 1, s));
        HIP_TRY(launch_tilt_reduce(grad, w, h, ea.grad64, s, ea.skip));
        HIP_TRY(launch_tilt_finish(ea.x64, ea.grad64, w, h, d, gamma, terms_d, ea.p, ea.terms, T_d, s, ea.skip));
        return OCTMC_OK;
    }
    bool enqueue_only() const override { return true; }
};

// Device memory of a stage-1 solve: the field, its gradient and the solver's
// vectors, sized for the finest level.
struct StageMem {
    DevMem mem;
    Solver sv;
    double* terms_d = nullptr;
    double* T_d = nullptr;
    float* disp = nullptr;
    float* grad = nullptr;
    int alloc(size_t na, size_t nth, int m)
    {
        terms_d = mem.get<double>(OCTMC_NTERMS);
        T_d = mem.get<double>(1);
        disp = mem.get<float>(2 * na * 3);
        grad = mem.get<float>(2 * na * 3);
        sv.m = m;
        double** vecs[] = {&sv.x, &sv.g, &sv.p, &sv.xt, &sv.xprev, &sv.sc, &sv.yc, &sv.gt};
        for (double** v : vecs) *v = mem.get<double>(nth);
        bool ok = terms_d && T_d && disp && grad;
        for (double** v : vecs) ok = ok && *v;
        for (int k = 0; k < m; ++k) {
            sv.S[k] = mem.get<double>(nth);
            sv.Y[k] = mem.get<double>(nth);
            ok = ok && sv.S[k] && sv.Y[k];
        }
        sv.xt32 = mem.get<float>(nth);
        ok = ok && sv.xt32;
        return ok ? OCTMC_OK : fail(OCTMC_E_OOM, "out of device memory (stage 1)");
    }
};

struct PinnedScratch {
    double* terms = nullptr;
    double* dots = nullptr;
    int alloc()
    {
        HIP_TRY(hipHostMalloc(&terms, OCTMC_NTERMS * 8, hipHostMallocDefault));
        HIP_TRY(hipHostMalloc(&dots, (kMaxDots + 1) * 8, hipHostMallocDefault));
        return OCTMC_OK;
    }
    ~PinnedScratch()
    {
        if (terms) (void)hipHostFree(terms);
        if (dots) (void)hipHostFree(dots);
    }
};

int check_theta_level(const octmc_pair* pair, int level)
{
    if (!pair) return fail(OCTMC_E_INVALID, "pair is NULL");
    if (level < 0 || level >= pair_nlev(pair)) return fail(OCTMC_E_INVALID, "no such pyramid level");
    return OCTMC_OK;
}

}  // namespace

int prealign_solve(octmc_pair* pair, double gamma, int iters, std::vector<double>& theta, octmc_report* rep,
                   hipStream_t s)
{
    const int L = pair_nlev(pair);
    int w0, h0, d0;
    OCTMC_TRY(octmc_pair_level_shape(pair, 0, &w0, &h0, &d0));
    const size_t na0 = (size_t)w0 * h0, nth0 = 2 * (size_t)(w0 + h0);
    octmc_params pr = pair_params(pair);
    pr.iters_per_level = iters;
    StageMem sm;
    OCTMC_TRY(sm.alloc(na0, nth0, pr.lbfgs_m));
    PinnedScratch hs;
    OCTMC_TRY(hs.alloc());
    const bool device_ls = !(pr.flags & OCTMC_HOST_LINE_SEARCH) && pr.lbfgs_m <= kLbMaxM;
    std::vector<double> th;
    int wc = 0, hc = 0;
    if (rep) *rep = octmc_report{};
    for (int l = L - 1; l >= 0; --l) {
        int w, h, d;
        OCTMC_TRY(octmc_pair_level_shape(pair, l, &w, &h, &d));
        th = th.empty() ? std::vector<double>(2 * (size_t)(w + h), 0.0) : upsample_theta(th, wc, hc, w, h);
        const size_t n = th.size();
        HIP_TRY(hipMemcpyAsync(sm.sv.x, th.data(), n * 8, hipMemcpyHostToDevice, s));
        sm.sv.n = n;
        StageEvaluator ev(pair, w, h, d, gamma, sm.terms_d, sm.T_d, sm.disp, sm.grad);
        LevelRun run{pair, l, &sm.sv, s, n, hs.terms, hs.dots, &ev};
        LevelStats st{};
        if (device_ls)
            OCTMC_TRY(run.run_device(pr, st));
        else
            OCTMC_TRY(run.run(pr, st));
        HIP_TRY(hipMemcpyAsync(th.data(), sm.sv.x, n * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (!std::isfinite(st.f_end)) return fail(OCTMC_E_NAN, "non-finite stage-1 objective");
        if (rep) {
            const int r = L - 1 - l;
            rep->iters[r] = st.iters;
            rep->evals[r] = st.evals;
            rep->ls_fail[r] = st.ls_fail;
            rep->eta[r] = 1.0;
            rep->f_start[r] = st.f_start;
            rep->f_end[r] = st.f_end;
            rep->nlevels = L - l;
        }
        wc = w;
        hc = h;
    }
    theta = th;
    return OCTMC_OK;
}

}  // namespace octmc

using namespace octmc;

extern "C" {

int octmc_prealign_eval(octmc_pair* pair, int32_t level, const double* theta, double gamma_tilt, double* terms,
                        double* tilt_term_out, double* grad_theta, void* stream)
{
    OCTMC_TRY(check_theta_level(pair, level));
    if (!theta || !terms) return fail(OCTMC_E_INVALID, "theta and terms are required");
    if (pair->busy.load()) return fail(OCTMC_E_BUSY, "pair is in use");
    if (!std::isfinite(gamma_tilt) || gamma_tilt < 0) return fail(OCTMC_E_INVALID, "gamma_tilt must be >= 0");
    HIP_TRY(hipSetDevice(pair_device(pair)));
    int w, h, d;
    OCTMC_TRY(octmc_pair_level_shape(pair, level, &w, &h, &d));
    const size_t na = (size_t)w * h, nth = 2 * (size_t)(w + h);
    DevMem mem;
    double* th_d = mem.get<double>(nth);
    double* gth_d = mem.get<double>(nth);
    double* terms_d = mem.get<double>(2 * OCTMC_NTERMS + 1);
    float* disp = mem.get<float>(2 * na * 3);
    float* grad = mem.get<float>(2 * na * 3);
    if (!th_d || !gth_d || !terms_d || !disp || !grad) return fail(OCTMC_E_OOM, "out of device memory (stage 1)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    StageEvaluator ev(pair, w, h, d, gamma_tilt, terms_d, terms_d + 2 * OCTMC_NTERMS, disp, grad);
    HIP_TRY(hipMemcpyAsync(th_d, theta, nth * 8, hipMemcpyHostToDevice, s));
    EvalArgs ea{pair, nullptr, terms_d + OCTMC_NTERMS, nullptr, nullptr, gth_d, level, 1};
    ea.x64 = th_d;
    OCTMC_TRY(ev.eval(ea, s));
    std::vector<double> out(2 * OCTMC_NTERMS + 1);
    HIP_TRY(hipMemcpyAsync(out.data(), terms_d, out.size() * 8, hipMemcpyDeviceToHost, s));
    if (grad_theta) HIP_TRY(hipMemcpyAsync(grad_theta, gth_d, nth * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (!std::isfinite(out[OCTMC_NTERMS + OCTMC_TERM_F])) return fail(OCTMC_E_NAN, "non-finite stage-1 objective");
    for (int q = 0; q < OCTMC_NTERMS; ++q) terms[q] = out[q];  // the field objective's terms, without T
    if (tilt_term_out) *tilt_term_out = out[2 * OCTMC_NTERMS];
    return OCTMC_OK;
}

int octmc_prealign(octmc_pair* pair, double gamma_tilt, int32_t iters_per_level, double* theta_out,
                   octmc_report* rep, void* stream)
{
    if (!pair || !theta_out) return fail(OCTMC_E_INVALID, "pair and theta_out are required");
    if (!std::isfinite(gamma_tilt) || gamma_tilt < 0) return fail(OCTMC_E_INVALID, "gamma_tilt must be >= 0");
    if (iters_per_level < 0) return fail(OCTMC_E_INVALID, "iters_per_level must be >= 0");
    int idle = 0;
    if (!pair->busy.compare_exchange_strong(idle, 1)) return fail(OCTMC_E_BUSY, "pair is in use");
    struct Unbusy {
        octmc_pair* p;
        ~Unbusy() { p->busy.store(0); }
    } ub{pair};
    HIP_TRY(hipSetDevice(pair_device(pair)));
    std::vector<double> th;
    OCTMC_TRY(prealign_solve(pair, gamma_tilt, iters_per_level, th, rep, static_cast<hipStream_t>(stream)));
    for (size_t q = 0; q < th.size(); ++q) theta_out[q] = th[q];
    return OCTMC_OK;
}

int octmc_pair_prealignment(const octmc_pair* pair, double* theta_out, float* dz_out, void* stream)
{
    if (!pair) return fail(OCTMC_E_INVALID, "pair is NULL");
    const std::vector<double>& th = pair_theta(pair);
    if (th.empty()) return fail(OCTMC_E_INVALID, "the pair was not created with OCTMC_PREALIGN");
    int w, h, d;
    OCTMC_TRY(octmc_pair_level_shape(pair, 0, &w, &h, &d));
    if (theta_out)
        for (size_t q = 0; q < th.size(); ++q) theta_out[q] = th[q];
    if (dz_out) {
        HIP_TRY(hipSetDevice(pair_device(pair)));
        hipStream_t s = static_cast<hipStream_t>(stream);
        DevMem mem;
        double* th_d = mem.get<double>(th.size());
        if (!th_d) return fail(OCTMC_E_OOM, "out of device memory");
        HIP_TRY(hipMemcpyAsync(th_d, th.data(), th.size() * 8, hipMemcpyHostToDevice, s));
        HIP_TRY(launch_tilt_expand(th_d, w, h, nullptr, dz_out, s));
        HIP_TRY(hipStreamSynchronize(s));  // th_d is freed on return
    }
    return OCTMC_OK;
}

int octmc_resample_axial(octmc_ctx* ctx, const octmc_shape* shape, const float* vol, const float* dz, float* out,
                         void* stream)
{
    if (!ctx || !shape || !vol || !dz || !out) return fail(OCTMC_E_INVALID, "NULL argument");
    if (shape->mem != OCTMC_MEM_HOST && shape->mem != OCTMC_MEM_DEVICE)
        return fail(OCTMC_E_INVALID, "unknown memory kind");
    const int w = shape->w, h = shape->h, d = shape->d;
    if (w < 1 || h < 1 || d < 1) return fail(OCTMC_E_SHAPE, "empty volume");
    const size_t na = (size_t)w * h, nv = na * d;
    if (nv * 4 >= (1ull << 31)) return fail(OCTMC_E_SHAPE, "volume larger than 2^31 bytes");
    HIP_TRY(hipSetDevice(ctx_device(ctx)));
    hipStream_t s = static_cast<hipStream_t>(stream);
    DevMem mem;
    const float *v = vol, *z = dz;
    if (shape->mem == OCTMC_MEM_HOST) {
        float* q = mem.get<float>(nv + na);
        if (!q) return fail(OCTMC_E_OOM, "out of device memory (input copies)");
        HIP_TRY(hipMemcpyAsync(q, vol, nv * 4, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(q + nv, dz, na * 4, hipMemcpyHostToDevice, s));
        v = q;
        z = q + nv;
    }
    HIP_TRY(launch_resample_z(v, z, na, d, out, s));
    if (!mem.p.empty()) HIP_TRY(hipStreamSynchronize(s));  // the copies are freed on return
    return OCTMC_OK;
}

}  // extern "C"
