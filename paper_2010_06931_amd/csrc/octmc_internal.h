// Internal declarations of the octmc HIP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/octmc.h"

namespace octmc {

// Error reporting: set the calling thread's last error (octmc_last_error) and
// return `code`.
int fail(int code, const std::string& msg);

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return ::octmc::fail(e_ == hipErrorOutOfMemory ? OCTMC_E_OOM : OCTMC_E_DEVICE,         \
                                 std::string(#expr) + ": " + hipGetErrorString(e_));               \
    } while (0)

#define OCTMC_TRY(expr)                                                                            \
    do {                                                                                           \
        int r_ = (expr);                                                                           \
        if (r_ != OCTMC_OK) return r_;                                                             \
    } while (0)

// A contiguous range of device memory handed out by bumping an offset (every
// allocation 256-byte aligned); nothing is freed before the whole range is.
struct Slab {
    char* base = nullptr;
    size_t size = 0;
    size_t used = 0;
    void* take(size_t bytes)
    {
        const size_t off = (used + 255) & ~(size_t)255;
        if (off > size || bytes > size - off) return nullptr;
        used = off + bytes;
        return base + off;
    }
};
inline size_t slab_bytes(size_t bytes) { return (bytes + 255) & ~(size_t)255; }

struct EvalView;

// One evaluation job: a pair at one of its pyramid levels.
struct EvalArgs {
    octmc_pair* pair;
    const float* disp;               // [2][na][3], or the first slot's [na][3] when disp_y is set
    double* terms;
    float* grad;
    const double* p = nullptr;       // search direction for the directional derivative (or null)
    double* grad64 = nullptr;        // float64 gradient for the solver (or null)
    int level = 0;
    int eta_mode = 1;                // 0: set the level's eta first (Eq. 10)
    const float* disp_y = nullptr;   // the second slot's [na][3] (null: disp + na * 3); needs with_struct =
                                     // false in eval_group, whose structural kernels read [2][na][3]
    bool axial = false;              // dx = dy = 0 everywhere (stage 1): the x, y partials are left at 0
    const EvalView* view = nullptr;  // the level's data, parameters and scratch; null: those of pair at level
    const int* skip = nullptr;       // device flag: when nonzero every kernel of the evaluation does nothing
    const double* x64 = nullptr;     // the solver's float64 point (x or the trial point), for evaluators
                                     // whose parameters are not the field itself (stage 1)
};

// The hot path over up to kMaxJobs jobs (distinct pairs, one storage type,
// any levels and sizes) in one launch per kernel, on stream s.  ev (4 events
// or null) brackets the three stages for timing.
int eval_group(const EvalArgs* ea, int n, hipStream_t s, hipEvent_t* ev = nullptr, bool with_struct = true);

// How the solver gets its evaluations: directly on its stream, or through a
// scheduler that groups the evaluations of several solvers.  eval() returns
// once the evaluation is ordered before any later work on s.
struct Evaluator {
    virtual ~Evaluator() = default;
    virtual int eval(const EvalArgs& ea, hipStream_t s) = 0;
    // true when eval() only enqueues the evaluation on s (no host work), so
    // that a solver may enqueue its iterations ahead with decisions taken on
    // the device
    virtual bool enqueue_only() const { return false; }
};

octmc_dtype pair_dtype(const octmc_pair* pair);
// A-scans (w h) of a pair's pyramid level.
int pair_level_ascans(const octmc_pair* pair, int level);
int validate_params(const octmc_params* p);
// params with levels = 0 (automatic) replaced by the level count for `shape`:
// the fewest levels whose coarsest level is at most kAutoCoarsest A-scans
// wide, stopping before an axis would fall below 4 samples
constexpr int kAutoCoarsest = 16;
octmc_params resolve_levels(const octmc_params& p, const octmc_shape& shape);
int validate_shape(const octmc_params* params, const octmc_shape* shape);

// Device bytes a pair (and its solve and merge) takes from a Slab.
size_t pair_footprint(const octmc_params& params, const octmc_shape& shape, bool have_octa, bool have_valid,
                      bool merged);

// The C-ABI operations with an optional slab (all device memory, including
// temporaries, comes from it), an evaluator and host scratch.
int pair_create_impl(octmc_ctx* ctx, const octmc_params* params, const octmc_shape* shape, const float* oct_x,
                     const float* oct_y, const float* octa_x, const float* octa_y, const float* enface_x,
                     const float* enface_y, const float* valid_x, const float* valid_y, hipStream_t s, Slab* slab,
                     octmc_pair** out);
int register_impl(octmc_pair* pair, float* disp_out, float* merged_oct, float* merged_octa, octmc_report* rep,
                  hipStream_t s, Evaluator* ev, Slab* slab, double* h_terms, double* h_dots);
int merge_impl(octmc_pair* pair, const float* disp, float* merged_oct, float* merged_octa, hipStream_t s,
               Slab* slab);
int ctx_device(const octmc_ctx* ctx);

constexpr int kMaxJobs = 8;     // jobs (pairs) per grouped launch

// Storage pitch of a volume level (samples from one A-scan's column to the
// next): the depth, plus one padding sample (a copy of the last) for an odd
// depth in 16-bit storage, so that every sample pair starts 32-bit aligned.
inline int storage_pitch(int d, octmc_dtype dt) { return (dt != OCTMC_F32 && (d & 1)) ? d + 1 : d; }
constexpr int kWavesPerBlock = 4;
constexpr int kRedBlock = 256;  // threads per block of the reduction kernels

// ---------------------------------------------------------------------------
// Hot path, step 1: per-A-scan structural residual sums (Eqs. 2-4 and their
// derivative), one wavefront per output A-scan.
struct StructJob {
    const void* sx;     // storage-type volume of the X-fast scan, [h][w][d]
    const void* sy;     // Y-fast
    const float* disp;  // [2][na][3]
    float* part;        // [na][8]: Lambda, Gamma^X (x,y,z), Gamma^Y (x,y,z), 0
    int w, h, d, na;
    int blk_begin;      // first block of this job in the grid
    uint32_t vol_bytes; // bytes of one volume (buffer range)
    float eps_h;        // pseudo-Huber parameter (Eq. 4)
    int dp;             // storage pitch: samples between neighbouring A-scans' columns (d or d + 1)
};
struct StructJobs {
    StructJob j[kMaxJobs];
    int n;
    const int* skip = nullptr;  // device flag: when nonzero the whole launch does nothing
};
// Blocks of one structural job: one 2 x 2 tile of A-scans per block, in 8
// bands of whole tile rows (one per XCD).
inline int struct_blocks(int w, int h) { return 8 * (((h + 1) / 2 + 7) / 8) * ((w + 1) / 2); }

// Hot path, step 0: sum of the displacements (for the mean term M), as one
// row of block partials per block (summed in a fixed order by its readers).
struct SumJob {
    const float* disp[2];  // [na][3] per slot
    double* blk;        // [nblk][4] block partials
    int na, blk_begin, nblk;
};
struct SumJobs {
    SumJob j[kMaxJobs];
    int n;
    const int* skip = nullptr;  // device flag: when nonzero the whole launch does nothing
};

// Hot path, steps 2-4: en face term, validity weight, combination with eta,
// regulariser, mean term, gradient and the deterministic global sums.
struct CombineJob {
    const float* part;   // [na][8] from the structural kernel
    const float* disp[2];  // [na][3] per slot
    float* grad;         // [2][na][3] or nullptr
    double* grad64;      // [2][na][3] float64 gradient (solver) or nullptr
    const float* ax;     // en face images [h][w]
    const float* ay;
    const float* vx;     // validity [h]
    const float* vy;     // validity [w]
    const double* sum_blk;  // [nsum][4] displacement-sum partials of step 0
    double* eta;         // level constant (read in mode 1, written in mode 0)
    const double* p;     // [2][na][3] search direction (float64) or nullptr
    double* blk;         // [nblk][8] block partials
    double* terms;       // [OCTMC_NTERMS] (mode 1)
    int w, h, d, na, blk_begin, nblk, nsum;
    int mode;            // 0: only set eta (Eq. 10); 1: full evaluation
    int orient;          // scan orientation of the two slots (bit 0: first, bit 1: second; 0 X-fast, 1 Y-fast)
    double delta0, eps_h, eps_r, alpha, gamma, wfb;
};
struct CombineJobs {
    CombineJob j[kMaxJobs];
    int n;
    const int* skip = nullptr;  // device flag: when nonzero the whole launch does nothing
};

// ---------------------------------------------------------------------------
// launchers (kernels_eval.hip)
hipError_t launch_sum(const SumJobs& jobs, int total_blocks, hipStream_t s);
// axial: every displacement has dx = dy = 0 (stage 1); the kernels then read
// the centre column alone and leave the x and y partials at 0
hipError_t launch_struct(const StructJobs& jobs, int total_blocks, octmc_dtype dt, hipStream_t s,
                         bool axial = false);
// per-A-scan combination (total_blocks) followed by the fixed-order final
// sums, one block per job
hipError_t launch_combine(const CombineJobs& jobs, int total_blocks, hipStream_t s);
// the structural partials of every volume pair of n volumes at one level,
// each volume resampled once (n = 3 or 4; float32 storage, or 16-bit storage
// at an even storage pitch dp: see struct_multi_supported); part[q] is pair
// q's [na][8] partial buffer, the pairs (P, Q), P < Q, in lexicographic
// order; skip (device flag, may be null): when nonzero the launch does nothing
bool struct_multi_supported(int n, int dp, octmc_dtype dt);
hipError_t launch_struct_multi(const void* const* vol, int n, const float* disp, float* const* part, int w, int h,
                               int d, int dp, uint32_t vol_bytes, float eps_h, octmc_dtype dt, hipStream_t s,
                               const int* skip = nullptr);

// preparation (kernels_prep.hip)
hipError_t launch_to_storage(const float* in, void* out, size_t n, octmc_dtype dt, hipStream_t s);
// float32 [na][d] -> storage type [na][dp] (dp >= d; samples d .. dp - 1 of
// every A-scan repeat sample d - 1)
hipError_t launch_to_storage_pitched(const float* in, void* out, int na, int d, int dp, octmc_dtype dt,
                                     hipStream_t s);
hipError_t launch_pyr3(const float* in, int w, int h, int d, float* out, hipStream_t s);
hipError_t launch_pyr2(const float* in, int w, int h, float* out, hipStream_t s);
hipError_t launch_pyr1(const float* in, int n, float* out, hipStream_t s);
hipError_t launch_enface_mean(const float* vol, int na, int d, float* out, hipStream_t s);
hipError_t launch_count_nonfinite(const float* v, size_t n, unsigned* counter, hipStream_t s);
hipError_t launch_copy_bscans(float* vol, int w, int h, int d, const int* src, int V, hipStream_t s);
hipError_t launch_upsample(const double* coarse, int wc, int hc, double* fine, int wf, int hf, hipStream_t s,
                           int nvol = 2);
// Stage 1, rough axial prealignment (kernels_prealign.hip, prealign.hip).
// theta: X-fast B-scans (h rows) then Y-fast B-scans (w columns), (offset,
// tilt) each.  launch_tilt_expand writes the [2][h][w][3] field (disp) and/or
// its axial component [2][h][w] (dz); launch_tilt_reduce the gradient with
// respect to theta from a field gradient; launch_resample_z the volume
// resampled along depth by a per-A-scan field.
// skip (device flag, may be null): when nonzero the launch does nothing.
hipError_t launch_tilt_expand(const double* theta, int w, int h, float* disp, float* dz, hipStream_t s,
                              const int* skip = nullptr);
hipError_t launch_tilt_reduce(const float* grad, int w, int h, double* gtheta, hipStream_t s,
                              const int* skip = nullptr);
// The tilt term T at theta (gamma_t: its weight, d: the level's depth) added
// to the stage-1 objective: terms_out = terms_in with F + T, T's gradient
// added to gtheta, terms_out[GP] = gtheta . p (0 without p), T into T_out
// (may be null).  One workgroup, fixed order of summation.
hipError_t launch_tilt_finish(const double* theta, double* gtheta, int w, int h, int d, double gamma_t,
                              const double* terms_in, const double* p, double* terms_out, double* T_out,
                              hipStream_t s, const int* skip = nullptr);
hipError_t launch_resample_z(const float* vol, const float* dz, size_t na, int d, float* out, hipStream_t s);
// stage-1 solve over the pair's pyramid (theta at the finest level)
int prealign_solve(octmc_pair* pair, double gamma, int iters, std::vector<double>& theta, octmc_report* rep,
                   hipStream_t s);
// octmc_pair_create with OCTMC_PREALIGN
int prealign_create(octmc_ctx* ctx, const octmc_params* params, const octmc_shape* shape, const float* oct_x,
                    const float* oct_y, const float* octa_x, const float* octa_y, const float* enface_x,
                    const float* enface_y, const float* valid_x, const float* valid_y, hipStream_t s,
                    octmc_pair** out);
// evaluation scratch of a pair whose finest level has na A-scans (runtime.hip)
int pair_alloc_scratch(octmc_pair* pair, size_t na, hipStream_t s);
// pair accessors (runtime.hip)
int pair_nlev(const octmc_pair* pair);
const octmc_params& pair_params(const octmc_pair* pair);
int pair_device(const octmc_pair* pair);
const std::vector<double>& pair_theta(const octmc_pair* pair);

// line search statistics of one pyramid level
struct LevelStats {
    int iters = 0, evals = 0, ls_fail = 0;
    double f_start = 0, f_end = 0;
};
// Safeguarded cubic step of the zoom phase of the strong Wolfe line search:
// the minimiser of the cubic through (a0, f0, g0) and (a1, f1, g1), kept 10 %
// inside the bracket (its midpoint when the cubic gives nothing usable).  The
// host line search and the device one share this code; FMA contraction is off
// so that both round every operation alike.
__host__ __device__ inline double cubic_min(double a0, double f0, double g0, double a1, double f1, double g1)
{
#pragma clang fp contract(off)
    const double lo = a1 < a0 ? a1 : a0, hi = a0 < a1 ? a1 : a0, span = hi - lo;
    const double mid = 0.5 * (a0 + a1);
    const double d1 = g0 + g1 - 3.0 * (f0 - f1) / (a0 - a1);
    const double disc = d1 * d1 - g0 * g1;
    if (!(disc >= 0)) return mid;
    const double d2 = (a1 > a0 ? 1.0 : -1.0) * sqrt(disc);
    const double den = g1 - g0 + 2.0 * d2;
    if (den == 0) return mid;
    const double a = a1 - (a1 - a0) * (g1 + d2 - d1) / den;
    if (!__builtin_isfinite(a) || a < lo + 0.1 * span || a > hi - 0.1 * span) return mid;
    return a;
}

// Segmentation-free en face projection (Sec. 2.3) of one scan; `scratch`
// holds enface_scratch_bytes(w, h, d) device bytes; `valid` is a device
// vector of nb = (V == 0 ? h : w) floats or NULL (all valid); `fixed` a host
// {p5, p95} or NULL; `count` device int[h*w] or NULL; `stats_host` host
// double[4] or NULL (p5, p95, threshold on the filtered volume, OCT
// threshold; valid once the stream has reached this point).
size_t enface_scratch_bytes(int w, int h, int d);
int enface_max_bscan();
hipError_t launch_enface_project(const float* oct, const float* octa, int w, int h, int d, int V,
                                 const float* valid, const double* fixed, float* out, int* count, double* stats_host,
                                 void* scratch, hipStream_t s);
// input validity of one OCTA volume (Sec. 2.2): means[nb] float64 scratch,
// valid[nb] float32 output, nb = h (V = 0) or w (V = 1)
hipError_t launch_validity(const float* vol, int w, int h, int d, int V, double* means, float* valid,
                           hipStream_t s);

// L-BFGS vector kernels (kernels_lbfgs.hip)
constexpr int kMaxDotVecs = 16;
constexpr int kMaxDots = 40;
struct DotSpec {
    const double* v[kMaxDotVecs];
    unsigned char a[kMaxDots], b[kMaxDots];
    int ndots;
    int gmax_vec;  // index of the vector whose max |.| is also reduced (-1: none)
};
// dot products (and the max |.|) in one pass: block partials, then a
// fixed-order sum of the partials in a second launch
hipError_t launch_multidot(const DotSpec& spec, size_t n, double* blk, double* out, hipStream_t s);
constexpr int kMaxComb = 20;
struct CombSpec {
    const double* v[kMaxComb];
    double c[kMaxComb];
    int nv;
};
hipError_t launch_lincomb(const CombSpec& spec, size_t n, double* out, hipStream_t s);

// ---------------------------------------------------------------------------
// The L-BFGS iteration with its decisions on the device (LevelRun::run_device).
// Single-thread controller kernels take, in float64 and in the same order of
// operations, the decisions LevelRun::run takes on the host, and every vector
// kernel and evaluation of an iteration is predicated on flags they set, so
// that the host can enqueue iterations ahead without waiting for them.  The
// history is kept oldest first; where the host swaps buffer pointers, the
// controllers rotate the device table vec[], so no vector is copied.
constexpr int kLbMaxM = 6;  // the 3 + 2 m vectors of an iteration's dot products fit one keyed pass
static_assert(3 + 2 * kLbMaxM <= kMaxDotVecs, "one keyed dot-product pass per iteration");
struct LbStatus {  // the leading part of LbState that the host reads back
    int status;    // 0 running; 1 gradient small; 2 line search failed; 3 step limit reached
    int stall;     // the line search needs more trials than its iteration holds (the host resumes it)
    int it, evals;
    int ls_done, ls_ok;
    double f, f_start;
};
static_assert(sizeof(LbStatus) == 40, "status block");
struct LbState {
    LbStatus h;
    int skip_iter;   // status || stall: the iteration's kernels do nothing
    int skip_trial;  // skip_iter || the line search ended: the trial and its evaluation do nothing
    int do_accept;   // the accept kernel commits the trial point (set on success, cleared by the next iteration)
    int resume;      // the host enqueues the trials of a stalled line search one at a time
    int m, count, has_cand, iters_max, ls_max_evals;
    int ls_phase, ls_i, ls_start;  // bracketing (0) or zoom (1); trial number; evaluations at its start
    int ncomb;
    double c1, c2;
    // [g, s_c, y_c, S_0 .. S_{m-1}, Y_0 .. Y_{m-1}]: gradient, candidate pair, history oldest first
    double* vec[3 + 2 * kLbMaxM];
    double SY[kLbMaxM][kLbMaxM];  // s_k . y_l (k <= l read)
    double YY[kLbMaxM][kLbMaxM];  // y_k . y_l
    // search direction p = c_g g + sum_k (c_s[k] S_k + c_y[k] Y_k), k oldest first; gp = g . p
    double c_g, c_s[kLbMaxM], c_y[kLbMaxM], gp;
    // strong Wolfe line search
    double a_try, a_prev, f_prev, g_prev, lo, flo, glo, hi, fhi, ghi, f0, g0;
};
struct LbInit {
    double* vec[3 + 2 * kLbMaxM];
    int m, iters_max, ls_max_evals;
    double c1, c2;
};
hipError_t launch_lb_init(LbState* st, const LbInit& in, const double* terms, hipStream_t s);
// The head of an iteration, each kernel skipped with skip_iter: the pending
// accept of the previous step (x = xt, g = gt, the candidate pair formed)
// and the dot products (and max |g|) over st->vec into the block partials
// blk, the history update and search direction, then p and the first trial
// point x + p (xt, and xt32 in float32).
hipError_t launch_lb_head(LbState* st, int m, size_t n, double* blk, double* x, const double* gt, double* p,
                          double* xt, float* xt32, hipStream_t s);
// a further trial point x + a_try p (skipped with skip_trial)
hipError_t launch_lb_trial(const LbState* st, const double* x, const double* p, size_t n, double* xt, float* xt32,
                           hipStream_t s);
// last = 1: the iteration's only trial slot (an unfinished search stalls)
hipError_t launch_lb_c2(LbState* st, const double* terms, int last, hipStream_t s);
// the pending accept alone (the level's last step)
hipError_t launch_lb_accept(const LbState* st, double* x, double* g, const double* xt, const double* gt, size_t n,
                            hipStream_t s);
// resume = 1: a stalled line search continues, one trial per host round trip; resume = 0: it ended
hipError_t launch_lb_resume(LbState* st, int resume, hipStream_t s);
hipError_t launch_trial(const double* x, const double* p, double alpha, size_t n, double* xt, float* xt32,
                        hipStream_t s);
hipError_t launch_accept(double* x, double* g, const double* xt, const double* gt, double* s_out,
                         double* y_out, size_t n, hipStream_t s);
hipError_t launch_to_f64(const float* in, double* out, size_t n, hipStream_t s);
hipError_t launch_to_f32(const double* in, float* out, size_t n, hipStream_t s);
hipError_t launch_fill_u32(unsigned* p, unsigned v, size_t n, hipStream_t s);

// merge (kernels_merge.hip)
hipError_t launch_density(const float* disp, int w, int h, unsigned long long* grid, hipStream_t s, int nvol = 2);
// merge of n volumes (2..kMaxVol): OCT and OCTA weights [n][na] from the
// densities and validities, then the weighted sum of the resampled volumes
constexpr int kMaxVol = 8;
struct MultiVols {
    const void* vol[kMaxVol];   // storage-type (or float32) volumes [h][w][d]
    const float* valid[kMaxVol];  // validity vectors (nullptr: no OCTA weights)
    int orient[kMaxVol];
    int n;
};
hipError_t launch_merge_weights_multi(const float* disp, int w, int h, const unsigned long long* grid,
                                      const MultiVols& mv, double kappa, double tau, float* wo, float* wa,
                                      hipStream_t s);
hipError_t launch_merge_volume_multi(const MultiVols& mv, octmc_dtype dt, const float* disp, const float* wts, int w,
                                     int h, int d, int dp, float* out, hipStream_t s);
hipError_t launch_merge_weights(const float* disp, int w, int h, const unsigned long long* grid,
                                const float* vx, const float* vy, double kappa, double tau, float4* wts,
                                hipStream_t s);
hipError_t launch_merge_volume(const void* vx_, const void* vy_, octmc_dtype dt, const float* disp,
                               const float4* wts, int which, int w, int h, int d, int dp, float* out, hipStream_t s);

}  // namespace octmc
