// Host-side types shared by the runtime translation units: the context, a
// pair's pyramid levels and scratch, the device L-BFGS solver state and its
// per-level loop.  Not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <deque>
#include <vector>

#include "octmc_internal.h"

struct octmc_ctx {
    int device;
    // device address of the evaluation scratch of octmc_eval_noalloc (the
    // file-scope array of runtime.hip on this device), resolved at creation
    void* noalloc_scratch = nullptr;
};

namespace octmc {

struct Level {
    int w = 0, h = 0, d = 0, na = 0;
    // storage pitch of sx / sy: samples from one A-scan's column to the next
    // (d, or d + 1 for an odd depth in 16-bit storage: the extra sample repeats
    // the last one, so that every sample pair starts 32-bit aligned)
    int dp = 0;
    void* sx = nullptr;
    void* sy = nullptr;
    float* ax = nullptr;
    float* ay = nullptr;
    float* vx = nullptr;
    float* vy = nullptr;
    uint32_t vol_bytes = 0;
};

// Everything one evaluation job reads besides its displacement: the level's
// volumes, en face images and validity, the objective's parameters, and the
// scratch its kernels write (per-A-scan partials [na][8] float32, the
// displacement-sum block rows [<= 256][4] and the combination block rows
// [nblk][8] float64) with the level's eta (one float64).
struct EvalView {
    Level L;
    octmc_dtype dtype = OCTMC_F32;
    const octmc_params* params = nullptr;
    float* part = nullptr;
    double* sum_blk = nullptr;
    double* comb_blk = nullptr;
    double* eta = nullptr;
    int orient = 2;
};

}  // namespace octmc

struct octmc_pair {
    octmc_ctx* ctx = nullptr;
    octmc_params params{};
    octmc_dtype dtype = OCTMC_F32;
    int nlev = 0;
    octmc::Level lev[OCTMC_MAX_LEVELS];
    float* octa[2] = {nullptr, nullptr};  // finest OCTA volumes (float32, invalid B-scans replaced)
    // evaluation scratch, sized for the finest level
    float* part = nullptr;      // [na0][8]
    double* sum_blk = nullptr;  // [256][4]
    unsigned* counters = nullptr;  // [8] non-finite input count
    double* comb_blk = nullptr; // [nblk0][8]
    double* eta = nullptr;      // [levels]
    double* terms = nullptr;    // [OCTMC_NTERMS] solver scratch
    double* dot_blk = nullptr;  // [512][kMaxDots + 1]
    double* dot_out = nullptr;  // [kMaxDots + 1]
    octmc::LbState* lb = nullptr;  // the device solver's state (LevelRun::run_device)
    std::vector<void*> owned;
    octmc::Slab* slab = nullptr;  // when set, all device memory comes from it
    std::atomic<int> busy{0};  // a solve holds the pair (taken by compare-and-swap)
    std::vector<double> theta;  // stage-1 offsets and tilts (created with OCTMC_PREALIGN)
    // scan orientation of the two slots (bit 0: first, bit 1: second; 0 =
    // X-fast, 1 = Y-fast): the validity direction and acquisition order
    int orient = 2;

    template <typename T>
    hipError_t alloc(T** p, size_t bytes)
    {
        void* q = nullptr;
        if (slab) {
            q = slab->take(bytes ? bytes : 16);
            if (!q) return hipErrorOutOfMemory;
            *p = static_cast<T*>(q);
            return hipSuccess;
        }
        hipError_t e = hipMalloc(&q, bytes ? bytes : 16);
        if (e == hipSuccess) {
            owned.push_back(q);
            *p = static_cast<T*>(q);
        }
        return e;
    }
    ~octmc_pair()
    {
        for (void* p : owned) (void)hipFree(p);
    }
};

namespace octmc {

// ---------------------------------------------------------------------------
// L-BFGS (textbook limited-memory BFGS with a strong Wolfe line search; the
// search direction is formed from the compact representation of the inverse
// Hessian approximation, which equals the two-loop recursion in exact
// arithmetic and needs one pass of dot products per iteration)

struct Solver {
    size_t n = 0;
    int m = 5;
    double *x = nullptr, *g = nullptr, *p = nullptr, *xt = nullptr, *xprev = nullptr;
    double *sc = nullptr, *yc = nullptr;  // candidate pair
    double* gt = nullptr;                 // gradient at the trial point
    double* S[8] = {};
    double* Y[8] = {};
    float* xt32 = nullptr;
};

struct LevelRun {
    octmc_pair* P;
    int level;
    Solver* sv;
    hipStream_t s;
    size_t n;
    double* h_terms;  // pinned host [OCTMC_NTERMS]
    double* h_dots;   // pinned host [kMaxDots + 1]
    Evaluator* ev;
    int evals = 0;

    // phi(alpha) = F(x + alpha p), dphi = g(x + alpha p) . p
    int trial(double alpha, double& f, double& dphi)
    {
        HIP_TRY(launch_trial(sv->x, sv->p, alpha, n, sv->xt, sv->xt32, s));
        EvalArgs ea{P, sv->xt32, P->terms, nullptr, sv->p, sv->gt, level, 1};
        ea.x64 = sv->xt;
        OCTMC_TRY(ev->eval(ea, s));
        HIP_TRY(hipMemcpyAsync(h_terms, P->terms, sizeof(double) * OCTMC_NTERMS, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        f = h_terms[OCTMC_TERM_F];
        dphi = h_terms[OCTMC_TERM_GP];
        ++evals;
        return OCTMC_OK;
    }

    // strong Wolfe line search; on success xt / gt hold the accepted point
    int line_search(double f0, double g0, int max_evals, int start_evals, double c1, double c2, bool& ok,
                    double& f_out)
    {
        ok = false;
        double a_prev = 0, f_prev = f0, g_prev = g0, a = 1.0;
        double lo, flo, glo, hi, fhi, ghi;
        for (int i = 1;; ++i) {
            if (evals - start_evals >= max_evals) return OCTMC_OK;
            double fa, ga;
            OCTMC_TRY(trial(a, fa, ga));
            if (fa > f0 + c1 * a * g0 || (i > 1 && fa >= f_prev)) {
                lo = a_prev; flo = f_prev; glo = g_prev;
                hi = a; fhi = fa; ghi = ga;
                break;
            }
            if (std::fabs(ga) <= -c2 * g0) {
                ok = true;
                f_out = fa;
                return OCTMC_OK;
            }
            if (ga >= 0) {
                lo = a; flo = fa; glo = ga;
                hi = a_prev; fhi = f_prev; ghi = g_prev;
                break;
            }
            a_prev = a; f_prev = fa; g_prev = ga;
            a = 2.0 * a;
        }
        for (;;) {
            if (evals - start_evals >= max_evals) return OCTMC_OK;
            const double aj = cubic_min(lo, flo, glo, hi, fhi, ghi);
            double fj, gj;
            OCTMC_TRY(trial(aj, fj, gj));
            if (fj > f0 + c1 * aj * g0 || fj >= flo) {
                hi = aj; fhi = fj; ghi = gj;
            } else {
                if (std::fabs(gj) <= -c2 * g0) {
                    ok = true;
                    f_out = fj;
                    return OCTMC_OK;
                }
                if (gj * (hi - lo) >= 0) {
                    hi = lo; fhi = flo; ghi = glo;
                }
                lo = aj; flo = fj; glo = gj;
            }
        }
    }

    // The same iteration as run(), with every decision taken on the device by
    // the k_lb_* controllers and every kernel of an iteration predicated on
    // their flags: the host enqueues kLbBatch iterations at a time, keeps two
    // batches in flight and reads a 40-byte status per batch.  Each iteration
    // holds one trial of its line search; a search that needs more stalls the
    // later iterations, which then do nothing, and the host drives its
    // remaining trials one round trip at a time, as run() does.  The first
    // iteration of a level, whose unit step along the scaled steepest descent
    // direction is the one least often accepted at once, is enqueued alone
    // and continued in the same way without stalling.
    static constexpr int kLbBatch = 4;
    int run_device(const octmc_params& pr, LevelStats& st)
    {
        LbState* S = P->lb;
        const int m = sv->m;
        HIP_TRY(launch_to_f32(sv->x, sv->xt32, n, s));
        {
            EvalArgs ea{P, sv->xt32, P->terms, nullptr, nullptr, sv->g, level, 0};
            ea.x64 = sv->x;
            OCTMC_TRY(ev->eval(ea, s));
        }
        LbInit in{};
        in.vec[0] = sv->g;
        in.vec[1] = sv->sc;
        in.vec[2] = sv->yc;
        for (int k = 0; k < m; ++k) {
            in.vec[3 + k] = sv->S[k];
            in.vec[3 + m + k] = sv->Y[k];
        }
        in.m = m;
        in.iters_max = pr.iters_per_level;
        in.ls_max_evals = pr.ls_max_evals;
        in.c1 = pr.c1;
        in.c2 = pr.c2;
        HIP_TRY(launch_lb_init(S, in, P->terms, s));
        LbStatus* hs = reinterpret_cast<LbStatus*>(h_dots);  // three 40-byte slots of the pinned buffer
        static_assert(3 * sizeof(LbStatus) <= (kMaxDots + 1) * sizeof(double), "status slots");
        struct Events {
            hipEvent_t e[2] = {nullptr, nullptr};
            ~Events()
            {
                for (hipEvent_t x : e)
                    if (x) (void)hipEventDestroy(x);
            }
        } evs;
        for (hipEvent_t& e : evs.e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        // the evaluation at the trial point and the line-search step after it
        auto eval_step = [&](int last) -> int {
            EvalArgs ea{P, sv->xt32, P->terms, nullptr, sv->p, sv->gt, level, 1};
            ea.skip = &S->skip_trial;
            ea.x64 = sv->xt;
            OCTMC_TRY(ev->eval(ea, s));
            HIP_TRY(launch_lb_c2(S, P->terms, last, s));
            return OCTMC_OK;
        };
        // one iteration: the previous step's accept with the dot products,
        // history update, direction and its first trial point, then the
        // evaluation there (its accept waits for the next iteration's head,
        // or for the accept after the level's last step)
        auto iteration = [&](int last) -> int {
            HIP_TRY(launch_lb_head(S, m, n, P->dot_blk, sv->x, sv->gt, sv->p, sv->xt, sv->xt32, s));
            OCTMC_TRY(eval_step(last));
            return OCTMC_OK;
        };
        auto read_now = [&](LbStatus& out) -> int {
            HIP_TRY(hipMemcpyAsync(&hs[2], S, sizeof(LbStatus), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            out = hs[2];
            return OCTMC_OK;
        };
        // the trials of a stalled line search (its accept is left pending)
        auto finish_search = [&](LbStatus& out) -> int {
            HIP_TRY(launch_lb_resume(S, 1, s));
            for (int r = 0;; ++r) {  // at most ls_max_evals trials end a search
                if (r > pr.ls_max_evals) return fail(OCTMC_E_DEVICE, "device line search did not end");
                HIP_TRY(launch_lb_trial(S, sv->x, sv->p, n, sv->xt, sv->xt32, s));
                OCTMC_TRY(eval_step(0));
                OCTMC_TRY(read_now(out));
                if (out.ls_done) break;
            }
            HIP_TRY(launch_lb_resume(S, 0, s));
            return OCTMC_OK;
        };
        LbStatus cur{};
        OCTMC_TRY(read_now(cur));
        if (cur.status == 0) {  // the first iteration, then its further trials one at a time
            OCTMC_TRY(iteration(0));
            OCTMC_TRY(read_now(cur));
            if (cur.status == 0 && !cur.ls_done) OCTMC_TRY(finish_search(cur));
        }
        struct Batch {
            int slot, k;
        };
        Batch q[2];
        int nq = 0, next = 0;
        int it_known = cur.it, inflight = 0;  // inflight: iterations enqueued after the status last read
        while (cur.status == 0) {
            while (nq < 2 && it_known + inflight < pr.iters_per_level) {
                const int k = std::min(kLbBatch, pr.iters_per_level - it_known - inflight);
                for (int i = 0; i < k; ++i) OCTMC_TRY(iteration(1));
                HIP_TRY(hipMemcpyAsync(&hs[next], S, sizeof(LbStatus), hipMemcpyDeviceToHost, s));
                HIP_TRY(hipEventRecord(evs.e[next], s));
                q[nq++] = Batch{next, k};
                next ^= 1;
                inflight += k;
            }
            if (nq == 0) break;  // every step the level allows is made (the status says so)
            const Batch b = q[0];
            q[0] = q[1];
            --nq;
            HIP_TRY(hipEventSynchronize(evs.e[b.slot]));
            cur = hs[b.slot];
            inflight -= b.k;
            it_known = cur.it;
            if (cur.status != 0) break;
            if (cur.stall) {  // the iterations enqueued after the stall do nothing
                HIP_TRY(hipStreamSynchronize(s));
                nq = 0;
                inflight = 0;
                OCTMC_TRY(finish_search(cur));
                it_known = cur.it;
            }
        }
        HIP_TRY(launch_lb_accept(S, sv->x, sv->g, sv->xt, sv->gt, n, s));  // the last step's, if pending
        OCTMC_TRY(read_now(cur));
        st.iters = cur.it;
        st.evals = cur.evals;
        st.f_start = cur.f_start;
        st.f_end = cur.f;
        st.ls_fail = cur.status == 2;
        evals = cur.evals;
        return OCTMC_OK;
    }

    int run(const octmc_params& pr, LevelStats& st)
    {
        const int m = sv->m;
        // initial evaluation: sets eta at the level's initial field (Eq. 10)
        HIP_TRY(launch_to_f32(sv->x, sv->xt32, n, s));
        {
            EvalArgs ea{P, sv->xt32, P->terms, nullptr, nullptr, sv->g, level, 0};
            ea.x64 = sv->x;
            OCTMC_TRY(ev->eval(ea, s));
        }
        HIP_TRY(hipMemcpyAsync(h_terms, P->terms, sizeof(double) * OCTMC_NTERMS, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        evals = 1;
        double f = h_terms[OCTMC_TERM_F];
        st.f_start = f;
        // history in chronological order (slot indices) and its dot products
        std::deque<int> order;
        double SY[8][8] = {}, YY[8][8] = {};  // SY[k][l] = s_k . y_l, YY[k][l] = y_k . y_l (slots)
        bool cand = false;
        int it = 0;
        while (it < pr.iters_per_level) {
            // one pass of dot products
            DotSpec ds{};
            int nv = 0;
            const int vg = nv++;
            ds.v[vg] = sv->g;
            int vs = -1, vy = -1;
            if (cand) {
                vs = nv++;
                ds.v[vs] = sv->sc;
                vy = nv++;
                ds.v[vy] = sv->yc;
            }
            int vS[8], vY[8];
            for (size_t k = 0; k < order.size(); ++k) {
                vS[k] = nv++;
                ds.v[vS[k]] = sv->S[order[k]];
                vY[k] = nv++;
                ds.v[vY[k]] = sv->Y[order[k]];
            }
            int nd = 0;
            auto dot = [&](int a, int b) {
                ds.a[nd] = (unsigned char)a;
                ds.b[nd] = (unsigned char)b;
                return nd++;
            };
            const int i_gg = dot(vg, vg);
            int i_sg[8], i_yg[8], i_syc[8], i_ycy[8];
            for (size_t k = 0; k < order.size(); ++k) {
                i_sg[k] = dot(vS[k], vg);
                i_yg[k] = dot(vY[k], vg);
                if (cand) {
                    i_syc[k] = dot(vS[k], vy);
                    i_ycy[k] = dot(vy, vY[k]);
                }
            }
            int i_csg = -1, i_cyg = -1, i_csy = -1, i_cyy = -1;
            if (cand) {
                i_csg = dot(vs, vg);
                i_cyg = dot(vy, vg);
                i_csy = dot(vs, vy);
                i_cyy = dot(vy, vy);
            }
            ds.ndots = nd;
            ds.gmax_vec = vg;
            HIP_TRY(launch_multidot(ds, n, P->dot_blk, P->dot_out, s));
            HIP_TRY(hipMemcpyAsync(h_dots, P->dot_out, sizeof(double) * (kMaxDots + 1), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            const double gg = h_dots[i_gg], gmax = h_dots[nd];
            // the new pair enters the memory only if it passes the curvature test
            std::vector<double> a_s(order.size()), b_y(order.size());
            for (size_t k = 0; k < order.size(); ++k) {
                a_s[k] = h_dots[i_sg[k]];
                b_y[k] = h_dots[i_yg[k]];
            }
            if (cand) {
                const double sy = h_dots[i_csy], yy = h_dots[i_cyy];
                if (sy > 1e-12 * yy && yy > 0) {
                    int slot;
                    if ((int)order.size() == m) {
                        slot = order.front();
                        order.pop_front();
                        a_s.erase(a_s.begin());
                        b_y.erase(b_y.begin());
                        // keep the dots of the remaining pairs with the candidate
                        for (size_t k = 0; k + 1 <= order.size(); ++k) {
                            i_syc[k] = i_syc[k + 1];
                            i_ycy[k] = i_ycy[k + 1];
                        }
                    } else {
                        std::vector<bool> used(m, false);
                        for (int q : order) used[q] = true;
                        slot = 0;
                        while (used[slot]) ++slot;
                    }
                    std::swap(sv->S[slot], sv->sc);
                    std::swap(sv->Y[slot], sv->yc);
                    for (size_t k = 0; k < order.size(); ++k) {
                        SY[order[k]][slot] = h_dots[i_syc[k]];
                        YY[order[k]][slot] = YY[slot][order[k]] = h_dots[i_ycy[k]];
                    }
                    SY[slot][slot] = sy;
                    YY[slot][slot] = yy;
                    order.push_back(slot);
                    a_s.push_back(h_dots[i_csg]);
                    b_y.push_back(h_dots[i_cyg]);
                }
                cand = false;
            }
            if (gmax <= 1e-10 * std::max(1.0, std::fabs(f))) break;
            double gp;
            const int c = (int)order.size();
            auto steepest = [&]() -> int {
                CombSpec cs{};
                cs.nv = 1;
                cs.v[0] = sv->g;
                cs.c[0] = -1.0 / gmax;
                HIP_TRY(launch_lincomb(cs, n, sv->p, s));
                gp = -gg / gmax;
                return OCTMC_OK;
            };
            if (c == 0) {
                OCTMC_TRY(steepest());
            } else {
                // H g = gamma g + S u + gamma Y v with v = -R^-1 a and
                // u = R^-T ((D + gamma Y'Y) R^-1 a - gamma b), R = upper(S'Y)
                const int nw = order.back();
                const double gamma = SY[nw][nw] / YY[nw][nw];
                std::vector<double> R(c * c, 0.0), t1(c), rhs(c), u(c);
                for (int k = 0; k < c; ++k)
                    for (int l = k; l < c; ++l) R[k * c + l] = SY[order[k]][order[l]];
                for (int k = c - 1; k >= 0; --k) {  // R t1 = a
                    double v = a_s[k];
                    for (int l = k + 1; l < c; ++l) v -= R[k * c + l] * t1[l];
                    t1[k] = v / R[k * c + k];
                }
                for (int k = 0; k < c; ++k) {
                    double v = SY[order[k]][order[k]] * t1[k];
                    for (int l = 0; l < c; ++l) v += gamma * YY[order[k]][order[l]] * t1[l];
                    rhs[k] = v - gamma * b_y[k];
                }
                for (int k = 0; k < c; ++k) {  // R' u = rhs
                    double v = rhs[k];
                    for (int l = 0; l < k; ++l) v -= R[l * c + k] * u[l];
                    u[k] = v / R[k * c + k];
                }
                CombSpec cs{};
                cs.nv = 1 + 2 * c;
                cs.v[0] = sv->g;
                cs.c[0] = -gamma;
                double hg = gamma * gg;
                for (int k = 0; k < c; ++k) {
                    cs.v[1 + 2 * k] = sv->S[order[k]];
                    cs.c[1 + 2 * k] = -u[k];
                    cs.v[2 + 2 * k] = sv->Y[order[k]];
                    cs.c[2 + 2 * k] = gamma * t1[k];
                    hg += u[k] * a_s[k] - gamma * t1[k] * b_y[k];
                }
                HIP_TRY(launch_lincomb(cs, n, sv->p, s));
                gp = -hg;
            }
            if (!(gp < 0)) {  // not a descent direction: drop the memory
                order.clear();
                OCTMC_TRY(steepest());
            }
            bool ok;
            double fn;
            const int start = evals;
            OCTMC_TRY(line_search(f, gp, pr.ls_max_evals, start, pr.c1, pr.c2, ok, fn));
            if (!ok) {
                st.ls_fail = 1;
                break;
            }
            HIP_TRY(launch_accept(sv->x, sv->g, sv->xt, sv->gt, sv->sc, sv->yc, n, s));
            cand = true;
            f = fn;
            ++it;
        }
        st.iters = it;
        st.evals = evals;
        st.f_end = f;
        return OCTMC_OK;
    }
};

struct DirectEvaluator final : Evaluator {
    int eval(const EvalArgs& ea, hipStream_t s) override { return eval_group(&ea, 1, s); }
    bool enqueue_only() const override { return true; }
};

}  // namespace octmc
