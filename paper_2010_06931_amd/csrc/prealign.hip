// Stage 1, rough axial prealignment (Fig. 1, Sec. 2.1 "optimization"): the
// objective of Eq. 1 restricted to axial displacements with one offset and
// one tilt per B-scan, plus the tilt normalisation T, minimised by L-BFGS on
// the factor-2 pyramid; and the axial resampling that turns its result into
// the prealigned volumes.
//
// The stage evaluates the pair's objective with the library's kernels at the
// field expanded from theta (kernels_prealign.hip) and reduces the field
// gradient back onto theta.  theta has 2 (h + w) values at a level of w x h
// A-scans, so its L-BFGS state lives on the host in float64; each
// evaluation moves 16 (h + w) bytes each way.
//
// T is defined only in earlier work that is not available.  Reading: a
// quadratic penalty on the sum of each scan's tilts,
//   T = sum_V gamma_t d n_f (n_f^2 - 1) / (24 n_b) (sum_b t_b)^2,
// which fixes the two degrees of freedom the data term cannot see (a common
// plane a x + b y added to both scans' fields) as M fixes the translations;
// a uniform tilt tau then costs gamma_t d N_A var_f tau^2 / 2.
#include <cmath>
#include <deque>
#include <vector>

#include "octmc_internal.h"

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

double tilt_term(const std::vector<double>& th, int w, int h, int d, double gamma, std::vector<double>* g)
{
    double T = 0.0;
    for (int V = 0; V < 2; ++V) {
        const int nb = V == 0 ? h : w, nf = V == 0 ? w : h;
        const size_t off = V == 0 ? 0 : 2 * (size_t)h;
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += th[off + 2 * b + 1];
        const double kap = gamma * d * (double)nf * ((double)nf * nf - 1.0) / (24.0 * nb);
        T += kap * s * s;
        if (g)
            for (int b = 0; b < nb; ++b) (*g)[off + 2 * b + 1] += 2.0 * kap * s;
    }
    return T;
}

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

// One stage-1 evaluation at one level: device buffers sized for the finest
// level, host copies of theta and of its gradient.
struct StageEval {
    octmc_pair* P;
    int level, w, h, d;
    double gamma;
    hipStream_t s;
    double* th_d;
    double* gth_d;
    double* terms_d;
    float* disp;
    float* grad;
    std::vector<double> terms = std::vector<double>(OCTMC_NTERMS);
    double T = 0.0;
    int evals = 0;

    int operator()(const std::vector<double>& th, double& f, std::vector<double>& g)
    {
        const size_t n = th.size();
        HIP_TRY(hipMemcpyAsync(th_d, th.data(), n * 8, hipMemcpyHostToDevice, s));
        HIP_TRY(launch_tilt_expand(th_d, w, h, disp, nullptr, s));
        EvalArgs ea{P, disp, terms_d, grad, nullptr, nullptr, level, 1};
        ea.axial = true;  // the field has dx = dy = 0; only its z gradient is used
        OCTMC_TRY(eval_group(&ea, 1, s));
        HIP_TRY(launch_tilt_reduce(grad, w, h, gth_d, s));
        g.resize(n);
        HIP_TRY(hipMemcpyAsync(g.data(), gth_d, n * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(terms.data(), terms_d, OCTMC_NTERMS * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        T = tilt_term(th, w, h, d, gamma, &g);
        f = terms[OCTMC_TERM_F] + T;
        ++evals;
        return std::isfinite(f) ? OCTMC_OK : fail(OCTMC_E_NAN, "non-finite stage-1 objective");
    }
};

double dotv(const std::vector<double>& a, const std::vector<double>& b)
{
    double s = 0.0;
    for (size_t k = 0; k < a.size(); ++k) s += a[k] * b[k];
    return s;
}

// L-BFGS with the two-loop recursion and a strong Wolfe line search (initial
// step 1, doubling bracket, safeguarded cubic zoom), float64 on the host; the
// same rules as the device solver of the 3-D registration.
int host_lbfgs(std::vector<double>& x, StageEval& fg, int m, int max_iter, int ls_max, double c1, double c2,
               LevelStats& st)
{
    const size_t n = x.size();
    std::vector<double> g, gt, xt(n), p(n), q(n);
    double f;
    OCTMC_TRY(fg(x, f, g));
    st.f_start = f;
    std::deque<std::vector<double>> S, Y;
    std::deque<double> rho;
    int it = 0;
    while (it < max_iter) {
        double gmax = 0.0;
        for (double v : g) gmax = std::max(gmax, std::fabs(v));
        if (gmax <= 1e-10 * std::max(1.0, std::fabs(f))) break;
        auto steepest = [&]() {
            for (size_t k = 0; k < n; ++k) p[k] = -g[k] / gmax;
        };
        if (S.empty()) {
            steepest();
        } else {
            q = g;
            std::vector<double> al(S.size());
            for (int c = (int)S.size() - 1; c >= 0; --c) {
                al[c] = rho[c] * dotv(S[c], q);
                for (size_t k = 0; k < n; ++k) q[k] -= al[c] * Y[c][k];
            }
            const double gamma = dotv(S.back(), Y.back()) / dotv(Y.back(), Y.back());
            for (size_t k = 0; k < n; ++k) q[k] *= gamma;
            for (size_t c = 0; c < S.size(); ++c) {
                const double bta = rho[c] * dotv(Y[c], q);
                for (size_t k = 0; k < n; ++k) q[k] += (al[c] - bta) * S[c][k];
            }
            for (size_t k = 0; k < n; ++k) p[k] = -q[k];
        }
        double g0 = dotv(g, p);
        if (!(g0 < 0)) {  // not a descent direction: drop the memory
            S.clear();
            Y.clear();
            rho.clear();
            steepest();
            g0 = dotv(g, p);
        }
        // strong Wolfe line search along p
        const int start = fg.evals;
        auto trial = [&](double a, double& fa, double& ga) -> int {
            for (size_t k = 0; k < n; ++k) xt[k] = x[k] + a * p[k];
            OCTMC_TRY(fg(xt, fa, gt));
            ga = dotv(gt, p);
            return OCTMC_OK;
        };
        bool ok = false;
        double fn = f;
        {
            double a_prev = 0, f_prev = f, g_prev = g0, a = 1.0;
            double lo = 0, flo = f, glo = g0, hi = 0, fhi = f, ghi = g0;
            bool bracket = false;
            for (int i = 1;; ++i) {
                if (fg.evals - start >= ls_max) break;
                double fa, ga;
                OCTMC_TRY(trial(a, fa, ga));
                if (fa > f + c1 * a * g0 || (i > 1 && fa >= f_prev)) {
                    lo = a_prev; flo = f_prev; glo = g_prev;
                    hi = a; fhi = fa; ghi = ga;
                    bracket = true;
                    break;
                }
                if (std::fabs(ga) <= -c2 * g0) {
                    ok = true;
                    fn = fa;
                    break;
                }
                if (ga >= 0) {
                    lo = a; flo = fa; glo = ga;
                    hi = a_prev; fhi = f_prev; ghi = g_prev;
                    bracket = true;
                    break;
                }
                a_prev = a; f_prev = fa; g_prev = ga;
                a = 2.0 * a;
            }
            while (bracket && !ok) {
                if (fg.evals - start >= ls_max) break;
                const double aj = cubic_min(lo, flo, glo, hi, fhi, ghi);
                double fj, gj;
                OCTMC_TRY(trial(aj, fj, gj));
                if (fj > f + c1 * aj * g0 || fj >= flo) {
                    hi = aj; fhi = fj; ghi = gj;
                } else {
                    if (std::fabs(gj) <= -c2 * g0) {
                        ok = true;
                        fn = fj;
                        break;
                    }
                    if (gj * (hi - lo) >= 0) {
                        hi = lo; fhi = flo; ghi = glo;
                    }
                    lo = aj; flo = fj; glo = gj;
                }
            }
        }
        if (!ok) {
            st.ls_fail = 1;
            break;
        }
        // the new pair enters the memory only if it passes the curvature test
        std::vector<double> sv(n), yv(n);
        for (size_t k = 0; k < n; ++k) {
            sv[k] = xt[k] - x[k];
            yv[k] = gt[k] - g[k];
        }
        const double sy = dotv(sv, yv), yy = dotv(yv, yv);
        if (sy > 1e-12 * yy && yy > 0) {
            if ((int)S.size() == m) {
                S.pop_front();
                Y.pop_front();
                rho.pop_front();
            }
            S.push_back(std::move(sv));
            Y.push_back(std::move(yv));
            rho.push_back(1.0 / sy);
        }
        x = xt;
        g = gt;
        f = fn;
        ++it;
    }
    st.iters = it;
    st.evals = fg.evals;
    st.f_end = f;
    return OCTMC_OK;
}

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
    DevMem mem;
    const size_t na0 = (size_t)w0 * h0, nth0 = 2 * (size_t)(w0 + h0);
    double* th_d = mem.get<double>(nth0);
    double* gth_d = mem.get<double>(nth0);
    double* terms_d = mem.get<double>(OCTMC_NTERMS);
    float* disp = mem.get<float>(2 * na0 * 3);
    float* grad = mem.get<float>(2 * na0 * 3);
    if (!th_d || !gth_d || !terms_d || !disp || !grad) return fail(OCTMC_E_OOM, "out of device memory (stage 1)");
    const octmc_params& pr = pair_params(pair);
    std::vector<double> th;
    int wc = 0, hc = 0;
    if (rep) *rep = octmc_report{};
    for (int l = L - 1; l >= 0; --l) {
        int w, h, d;
        OCTMC_TRY(octmc_pair_level_shape(pair, l, &w, &h, &d));
        th = th.empty() ? std::vector<double>(2 * (size_t)(w + h), 0.0) : upsample_theta(th, wc, hc, w, h);
        StageEval fg{pair, l, w, h, d, gamma, s, th_d, gth_d, terms_d, disp, grad};
        LevelStats st{};
        OCTMC_TRY(host_lbfgs(th, fg, pr.lbfgs_m, iters, pr.ls_max_evals, pr.c1, pr.c2, st));
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
    if (!std::isfinite(gamma_tilt) || gamma_tilt < 0) return fail(OCTMC_E_INVALID, "gamma_tilt must be >= 0");
    HIP_TRY(hipSetDevice(pair_device(pair)));
    int w, h, d;
    OCTMC_TRY(octmc_pair_level_shape(pair, level, &w, &h, &d));
    const size_t na = (size_t)w * h, nth = 2 * (size_t)(w + h);
    DevMem mem;
    double* th_d = mem.get<double>(nth);
    double* gth_d = mem.get<double>(nth);
    double* terms_d = mem.get<double>(OCTMC_NTERMS);
    float* disp = mem.get<float>(2 * na * 3);
    float* grad = mem.get<float>(2 * na * 3);
    if (!th_d || !gth_d || !terms_d || !disp || !grad) return fail(OCTMC_E_OOM, "out of device memory (stage 1)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    StageEval fg{pair, level, w, h, d, gamma_tilt, s, th_d, gth_d, terms_d, disp, grad};
    std::vector<double> th(theta, theta + nth), g;
    double f;
    OCTMC_TRY(fg(th, f, g));
    for (int q = 0; q < OCTMC_NTERMS; ++q) terms[q] = fg.terms[q];
    if (tilt_term_out) *tilt_term_out = fg.T;
    if (grad_theta)
        for (size_t q = 0; q < nth; ++q) grad_theta[q] = g[q];
    return OCTMC_OK;
}

int octmc_prealign(octmc_pair* pair, double gamma_tilt, int32_t iters_per_level, double* theta_out,
                   octmc_report* rep, void* stream)
{
    if (!pair || !theta_out) return fail(OCTMC_E_INVALID, "pair and theta_out are required");
    if (!std::isfinite(gamma_tilt) || gamma_tilt < 0) return fail(OCTMC_E_INVALID, "gamma_tilt must be >= 0");
    if (iters_per_level < 0) return fail(OCTMC_E_INVALID, "iters_per_level must be >= 0");
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
