// Internal declarations of the octmc HIP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/octmc.h"

namespace octmc {

constexpr int kMaxJobs = 8;     // jobs (pairs) per grouped launch
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
};
struct StructJobs {
    StructJob j[kMaxJobs];
    int n;
};

// Hot path, step 0: sum of the displacements (for the mean term M).
struct SumJob {
    const float* disp;  // [2][na][3]
    double* blk;        // [nblk][4] block partials
    unsigned* counter;  // last-block counter (0 between launches)
    double* out;        // [3]
    int na, blk_begin, nblk;
};
struct SumJobs {
    SumJob j[kMaxJobs];
    int n;
};

// Hot path, steps 2-4: en face term, validity weight, combination with eta,
// regulariser, mean term, gradient and the deterministic global sums.
struct CombineJob {
    const float* part;   // [na][8] from the structural kernel
    const float* disp;   // [2][na][3]
    float* grad;         // [2][na][3] or nullptr
    double* grad64;      // [2][na][3] float64 gradient (solver) or nullptr
    const float* ax;     // en face images [h][w]
    const float* ay;
    const float* vx;     // validity [h]
    const float* vy;     // validity [w]
    const double* sumd;  // [3]
    double* eta;         // level constant (read in mode 1, written in mode 0)
    const double* p;     // [2][na][3] search direction (float64) or nullptr
    double* blk;         // [nblk][8]
    unsigned* counter;
    double* terms;       // [OCTMC_NTERMS] (mode 1)
    int w, h, d, na, blk_begin, nblk;
    int mode;            // 0: only set eta (Eq. 10); 1: full evaluation
    double delta0, eps_h, eps_r, alpha, gamma, wfb;
};
struct CombineJobs {
    CombineJob j[kMaxJobs];
    int n;
};

// ---------------------------------------------------------------------------
// launchers (kernels_eval.hip)
hipError_t launch_sum(const SumJobs& jobs, int total_blocks, hipStream_t s);
hipError_t launch_struct(const StructJobs& jobs, int total_blocks, octmc_dtype dt, hipStream_t s);
hipError_t launch_combine(const CombineJobs& jobs, int total_blocks, hipStream_t s);

// preparation (kernels_prep.hip)
hipError_t launch_to_storage(const float* in, void* out, size_t n, octmc_dtype dt, hipStream_t s);
hipError_t launch_pyr3(const float* in, int w, int h, int d, float* out, hipStream_t s);
hipError_t launch_pyr2(const float* in, int w, int h, float* out, hipStream_t s);
hipError_t launch_pyr1(const float* in, int n, float* out, hipStream_t s);
hipError_t launch_enface_mean(const float* vol, int na, int d, float* out, hipStream_t s);
hipError_t launch_count_nonfinite(const float* v, size_t n, unsigned* counter, hipStream_t s);
hipError_t launch_copy_bscans(float* vol, int w, int h, int d, const int* src, int V, hipStream_t s);
hipError_t launch_upsample(const double* coarse, int wc, int hc, double* fine, int wf, int hf, hipStream_t s);

// L-BFGS vector kernels (kernels_lbfgs.hip)
constexpr int kMaxDotVecs = 16;
constexpr int kMaxDots = 40;
struct DotSpec {
    const double* v[kMaxDotVecs];
    unsigned char a[kMaxDots], b[kMaxDots];
    int ndots;
    int gmax_vec;  // index of the vector whose max |.| is also reduced (-1: none)
};
hipError_t launch_multidot(const DotSpec& spec, size_t n, double* blk, unsigned* counter, double* out,
                           hipStream_t s);
constexpr int kMaxComb = 20;
struct CombSpec {
    const double* v[kMaxComb];
    double c[kMaxComb];
    int nv;
};
hipError_t launch_lincomb(const CombSpec& spec, size_t n, double* out, hipStream_t s);
hipError_t launch_trial(const double* x, const double* p, double alpha, size_t n, double* xt, float* xt32,
                        hipStream_t s);
hipError_t launch_accept(double* x, double* g, const double* xt, const double* gt, double* s_out,
                         double* y_out, size_t n, hipStream_t s);
hipError_t launch_to_f64(const float* in, double* out, size_t n, hipStream_t s);
hipError_t launch_to_f32(const double* in, float* out, size_t n, hipStream_t s);
hipError_t launch_fill_u32(unsigned* p, unsigned v, size_t n, hipStream_t s);

// merge (kernels_merge.hip)
hipError_t launch_density(const float* disp, int w, int h, unsigned long long* grid, hipStream_t s);
hipError_t launch_merge_weights(const float* disp, int w, int h, const unsigned long long* grid,
                                const float* vx, const float* vy, double kappa, double tau, float4* wts,
                                hipStream_t s);
hipError_t launch_merge_volume(const void* vx_, const void* vy_, octmc_dtype dt, const float* disp,
                               const float4* wts, int which, int w, int h, int d, float* out, hipStream_t s);

}  // namespace octmc
