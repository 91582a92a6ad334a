// Launch wrappers of the HIP kernels (one per pass family), instantiated for float and
// double in the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace psara {

struct LaunchArgs {
  const ProbDesc* descs;   // device array of problem descriptors
  const int4* items;       // device work list, one entry per workgroup
  int nitems;
  hipStream_t stream;
  int max_n = 0;           // largest image side among the launch's problems (0: not known)
  int ana_wide = 1;        // the analysis tilings among them: kAnaWide | kAnaAllBases bits
  int grid_ce = kChunkEntries;   // largest gridding chunk among them (entries staged per workgroup)
};

// P1 modes (the TV modes are Algorithm 3's primal steps: the data term enters as its gradient,
// held where Algorithm 1 holds Re phi^dagger B, and the row FFT that follows takes S_new)
enum PrimalMode { PM_CONSTRAINED = 0, PM_INIT = 1, PM_UNCONSTRAINED = 2, PM_TV_CONSTRAINED = 3,
                  PM_TV_UNCONSTRAINED = 4 };
__host__ __device__ constexpr bool pm_constrained(int m) { return m == PM_CONSTRAINED || m == PM_TV_CONSTRAINED; }
__host__ __device__ constexpr bool pm_positive_I(int m) {
  return m == PM_INIT || m == PM_UNCONSTRAINED || m == PM_TV_UNCONSTRAINED;
}
__host__ __device__ constexpr bool pm_tv(int m) { return m == PM_TV_CONSTRAINED || m == PM_TV_UNCONSTRAINED; }
// analysis modes
enum AnalysisMode { AM_DUAL = 0, AM_STORE = 1, AM_REWEIGHT = 2, AM_OBJECTIVE = 3, AM_MOMENTS = 4, AM_MAXABS = 5 };
// de-grid modes
// DG_STOKES: per Stokes map, Phi S - Y L^{-1} (the residual of Algorithm 3's data term)
enum DegridMode { DG_DUAL = 0, DG_FORWARD = 1, DG_RESIDUAL = 2, DG_STOKES = 3 };
// grid modes (GR_STOKES: the rows are per Stokes map already, no mixing)
enum GridMode { GR_DUAL = 0, GR_PLAIN = 1, GR_STOKES = 2 };

// pass 2 (P8) takes src_slot as the factor mode of the gridded values: 0 the factor the grid
// pass stored, 1 the l2-ball factor of the fused pass's partials, 2 one
template <typename R> void launch_fft(int pass, const LaunchArgs& a, int cells, int src_slot, int dst_slot);
template <typename R> void launch_primal_fft(int mode, const LaunchArgs& a, int cells);
// P9 of one iteration with P1 and P4 of the next (row work list)
template <typename R> void launch_fused_rows(int mode, const LaunchArgs& a, int cells);
template <typename R> void launch_degrid(int mode, const LaunchArgs& a, int max_ts, int taps, int src_slot, int out_slot);
template <typename R> void launch_grid(int mode, const LaunchArgs& a, int taps, int src_slot, int use_cfac);
// P6 + P7 of an iteration in one pass over the gridding work list (mode GR_DUAL: de-grid with
// the dual B step, then grid Bv; GR_STOKES: Algorithm 3's residual, then grid it); the column
// inverse FFT after it takes factor mode 1 (GR_DUAL) or 2 (GR_STOKES)
template <typename R> void launch_degrid_grid(int mode, const LaunchArgs& a, int taps, int src_slot, int out_slot);
template <typename R> void set_grid_kernel_limits(int max_ts, int taps);
void hip_check(hipError_t e, const char* what);
template <typename R> void launch_primal(int mode, const LaunchArgs& a);
template <typename R> void launch_analysis(int mode, int level, const LaunchArgs& a, int src_slot, int out_slot);
template <typename R> void launch_dirac(int mode, const LaunchArgs& a, int src_slot, int out_slot);
template <typename R> void launch_synthesis(int level, int coarsest, const LaunchArgs& a, int src_coef, int dst_slot);
// items {prob, tile, part, mask of bases}: part 0 writes dst_slot, part 1 dst_slot2
template <typename R> void launch_synthesis_final(const LaunchArgs& a, int src_coef, int dst_slot, int add_dirac,
                                                  int dst_slot2);
template <typename R> void launch_coarse(const LaunchArgs& a);
template <typename R> int coarse_level(int n, int levels);

// reductions and small utility kernels (items: {prob, block, -, -})
template <typename R> void launch_relvar(const LaunchArgs& a);
template <typename R> void launch_img_sumsq(const LaunchArgs& a, int slot, int channel, int scalar);
template <typename R> void launch_npcount(const LaunchArgs& a);
template <typename R> void launch_img_dot(const LaunchArgs& a, int xs, int ys);
template <typename R> void launch_img_scale(const LaunchArgs& a, int dst, int src, int scalar);
template <typename R> void launch_fill(void* p, size_t count, hipStream_t s);
// TV priors (items: {prob, block of 256 pixels, -, partial index}): the dual step of
// Algorithm 3 on X, Psi A into IMG_PSIA, and the prior's value of IMG_S into region 0 partials
template <typename R> void launch_tv_dual(const LaunchArgs& a);
template <typename R> void launch_tv_synth(const LaunchArgs& a);
template <typename R> void launch_tv_objective(const LaunchArgs& a);
// finalise: one workgroup per problem sums PART_GEN partials into scal[scalar]
void launch_finalize(const ProbDesc* descs, int nprob, int region, int count, int scalar, hipStream_t s);
void launch_finalize_zeta(const ProbDesc* descs, int nprob, hipStream_t s);
// adaptive stopping: count the chunk's iterations, halt the problems whose criteria hold, and
// write the number still running to active[0]
void launch_stop_decide(const ProbDesc* descs, int nprob, int chunk, int* active, hipStream_t s);
// scal[scalar] = max of the first entries of `count` pairs of generic region q
void launch_finalize_max(const ProbDesc* descs, int nprob, int q, int count, int scalar, hipStream_t s);
template <typename R> void launch_scale(void* p, size_t count, double factor, hipStream_t s);
// device-pointer data and image transfers (psara_set_data_dev, psara_get_image_dev)
void launch_nonfinite(const double* y, size_t n, int* bad, hipStream_t s);
template <typename R> void launch_gather_rows(const double* y, const int* perm, void* out, long long M, hipStream_t s);
template <typename R> void launch_to_double(const void* src, double* dst, size_t n, hipStream_t s);

}  // namespace psara
