// Host engine of one solve (or one member of a batch): device memory, work lists and
// the pass sequence, for one real type R (float: FP32 bulk with FP64 reductions; double).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <stdexcept>
#include <string>
#include <vector>

#include "common.hpp"
#include "error.hpp"
#include "launch.hpp"
#include "psara.h"

namespace psara {

void hip_check(hipError_t e, const char* what);

// Sorted visibility layout and tile binning of one uv coverage (precision independent).
struct Geometry {
  int n = 0, K = 0, T = 0, ts = 0, nts = 0, ntsg = 0;
  int64_t M = 0;
  double beta = 0.0;
  std::vector<int64_t> perm;      // sorted position -> caller index
  std::vector<int> k0;            // packed window starts (k1 << 16 | k2), sorted order
  std::vector<double> frac;       // (f1, f2) per sorted visibility
  std::vector<int> own_ptr;       // per tile: range of visibilities whose window starts there
  std::vector<int> row_beg, row_end;     // per gridding tile: its rows (window start in it), [beg, end)
  // gridding work: runs of a tile's rows sharing one window start (at most kRunMax long),
  // grouped into chunks of at most kChunkEntries entries; every chunk writes its tile and
  // the tile's halo to its own partial slot, summed when the column inverse FFT loads them
  std::vector<int> run_pack;             // per run: pack_run(entry offset in its chunk, length, window start in the tile)
  std::vector<int4> chunks;              // {tile, first run, end run, partial slot}
  std::vector<int2> chunk_ent;           // row range [lo, hi) each chunk covers
  std::vector<int2> tile_slots;          // per gridding tile {first partial slot, count}
  std::vector<int> slot_box;             // per slot: the region cells its chunk covers (pack_box)
  std::vector<int> tile_box;             // per gridding tile: the union of its slots' boxes
  std::vector<int> small_ids;            // chunks of at most kSmallChunk entries, heaviest first
  int n_slots = 0;
  int chunk_entries = kChunkEntries;     // the chunk size the runs and chunks were cut for
};

Geometry build_geometry(int n, int64_t M, const double* uv, int alpha, int T);
// (Re)cuts the gridding lists of a geometry into runs and chunks of at most chunk_entries entries.
void build_grid_chunks(Geometry& g, int chunk_entries);

// Launch shapes of a solve that the autotuner chooses among (they change the summation order of
// the gridding and the de-gridding norm, not what is computed).
struct Tuning {
  int grid_chunk = kChunkEntries;   // gridding entries per workgroup: 256, 512 or 1024
  int degrid_item = kDegridItem;    // visibilities per de-gridding workgroup: 64 .. 1024
  int ana_wide = 1;                 // analysis tiling: kAnaWide | kAnaAllBases bits (0 .. 3)
  int fft_cells = 0;                // grid cells per FFT workgroup (0: max(512, K)); 512, 1024, 2048
};
// Throws Error(PSARA_EINVAL) for a tuning outside those ranges or with fft_cells below the side K.
void check_tuning(const Tuning& t, int K);

// Work lists of the passes; every item names its problem (index into the descriptor array).
//   ana[l], syn[l]     SARA analysis / synthesis of level l for every level (non-dual uses)
//   ana_d[l], syn_d[l] the same restricted to the levels below each problem's fused coarse level
//   coarse             {prob, wavelet (-1: an empty place), Stokes channel, first coarse level}
//   synfinal           {prob, tile, 0, mask of every basis}
//   synsplit           the same with the bases of each tile split over two items {prob, tile, part,
//                      mask} of about equal filter work (one item per tile below two bases)
struct ItemSet {
  std::vector<int4> img, rows, cols, p6, p7, p7f, dirac, synfinal, synsplit, coarse;
  std::vector<int4> ana[kMaxLevels + 1], syn[kMaxLevels + 1];
  std::vector<int4> ana_d[kMaxLevels + 1], syn_d[kMaxLevels + 1];
};
void add_operator_items(ItemSet& S, int prob, const Geometry& g, int cells, int rcells, int dg_item, int* n_p6);
void add_prior_items(ItemSet& S, int prob, int n, int levels, int nwav, const int* wav_len, bool fp64, int c_level,
                     int ana_wide, int* n_ana_parts);

struct DevItems {
  int4* ptr = nullptr;
  int count = 0;
};

// The device work lists and launch shapes of one set of problems (one solve, or a batch of
// solves that share a precision and a tap count) that the iteration's pass sequence runs on.
struct PassLists {
  const ProbDesc* descs = nullptr;
  DevItems img, rows, cols, p6, p7, p7f, synfinal, coarse;
  DevItems ana_d[kMaxLevels + 1], syn_d[kMaxLevels + 1];
  int cells = 512, rcells = 512;   // FFT cells per workgroup of the column / row passes
  int max_ts = 16, taps = 8, max_levels = 0;
  int max_n = 0;                   // largest image side among the problems
  int ana_wide = 1;                // the problems' analysis tilings (kAnaWide | kAnaAllBases bits)
  int grid_ce = kChunkEntries;     // largest gridding chunk among the problems
  bool sparse = false;             // every problem has a wavelet prior (P2/P3 run)
  bool tv = false;                 // the problems carry a TV prior (Algorithm 3)
};

// `count` Algorithm-1 iterations of every problem in L: P1+P4, then per iteration P2/P3 on s1
// concurrently with P5..P8 on s0, joined back into s0, and P9 fused with the next iteration's
// P1+P4 (the last iteration ends with P9 alone, so the state between calls is the same as after
// `count` separate iterations).
template <typename R>
void launch_iterations(const PassLists& L, int mode, int count, hipStream_t s0, hipStream_t s1, hipEvent_t fork,
                       hipEvent_t join);
template <typename R>
void launch_sara_dual(const PassLists& L, hipStream_t s);   // P2 + P3 with the fused coarse levels

template <typename R>
struct Engine {
  Engine(const Geometry& g, hipStream_t stream);
  ~Engine();
  Engine(const Engine&) = delete;
  Engine& operator=(const Engine&) = delete;

  void set_data(const double* Y_sorted, double eps);
  // Y in device memory in the caller's row order (M x 4 complex doubles): false (Y unchanged) if
  // a value is not finite; returns when the caller's buffer is no longer read
  bool set_data_dev(const double* Y_dev, double eps);
  // per sorted visibility the 4 x 4 complex row mixing L D_m^T (32 doubles, row-major [s][j],
  // interleaved re, im), or NULL for the fixed L; the iteration state is reset
  void set_mixing(const double* mix_sorted);
  void set_prior(uint32_t mask, int levels, const double* weights, double gamma);
  // TV (kind 1) or l1 + TV (kind 2) prior of Algorithm 3 with per-Stokes weights
  void set_prior_tv(int kind, const double* tv_weight, const double* l1_weight);
  bool is_tv() const { return h_.tv_kind != 0; }
  void set_steps(double tau, double r1, double r2, double r3);
  void zero_state();
  void run(int mode, int iters);          // graph replay
  void capture(int mode, int iters);      // capture the graphs run(mode, iters) replays (no work launched)
  // Bytes of the iteration's scratch buffers: the gridding partial slots, then (at a 256-byte
  // boundary) the FP64 partial sums.
  size_t scratch_bytes() const;
  // `iters` iterations by direct launches with those buffers in caller-provided device memory
  // (scr, at least scratch_bytes()), allocating nothing; the context's own buffers are used
  // again afterwards.  Returns when the iterations are done.
  void run_in_scratch(int mode, int iters, void* scr, size_t cap);
  void run_eager(int mode, int iters);    // direct launches
  // Up to max_iters iterations, checking the stopping criteria stop = {theta, rel_var, np_max}
  // on the device after every check_every of them; returns the iterations run.
  int run_adaptive(int mode, int max_iters, int check_every, const double* stop);
  // clear the halt flag and counter, store the criteria and a device-side iteration bound
  // (0: none; the host bounds the run instead)
  void stop_begin(const double* stop, int max_iters = 0);
  void stop_poll(bool* halted, int* iters);   // the halt flag and the iterations counted so far
  int stop_end();                       // iterations run by the adaptive run; clears the halt flag
  void report(psara_report* r);
  double coef_std();
  double data_max_coef();              // max |Psi^dagger Re phi^dagger Y|
  void set_gamma(double gamma);        // rescale the thresholds gamma W to a new gamma
  void reweight(double delta);
  double opnorm(int max_iter, double rtol, int* iters_out);
  void apply_phi(const double* S, double* Y);
  void apply_phi_adjoint(const double* B, double* S);
  void apply_psi_adjoint(const double* S, double* A);
  void apply_psi(const double* A, double* S);
  void get_state(double* buf);
  void set_state(const double* buf);
  void get_img(int slot, double* dst, int comps);
  void get_img_dev(int slot, double* dst_dev, int comps);   // into device memory; returns when written
  void profile(int mode, int iters, double* ms);
  size_t coef_elems() const { return coef_elems_; }
  const Tuning& tuning() const { return tuning_; }
  int fft_cells() const { return cells_; }
  // new launch shapes: the gridding lists are cut again, the work lists rebuilt, the partial
  // sums and slots reallocated and the graphs dropped; the iteration state is kept
  void set_tuning(const Tuning& t);
  size_t device_bytes() const { return bytes_; }
  const ProbDesc& desc() const { return h_; }
  hipStream_t stream() const { return s0_; }
  const Geometry& geometry() const { return geo_; }
  int c_level() const { return c_level_; }
  bool has_prior() const { return h_.coef[COEF_A] != nullptr && h_.nwav > 0; }
  void sync() { sync_desc(); }

  // passes (stream 0 by default)
  void p1(int mode, hipStream_t s = nullptr);
  void p2(hipStream_t s = nullptr);
  void p3(int src_coef, int dst_slot, int add_dirac, hipStream_t s = nullptr);
  void p23(hipStream_t s = nullptr);   // the iteration's SARA branch: P2 and P3 with fused coarse levels
  void p4(int src, hipStream_t s = nullptr);
  void p5(hipStream_t s = nullptr);
  void p6(int mode, int src, int out, hipStream_t s = nullptr);
  void p7(int mode, int src, int use_cfac, hipStream_t s = nullptr);
  void p8(hipStream_t s = nullptr);
  void p9(int dst, hipStream_t s = nullptr);

 private:
  template <typename T> T* dalloc(size_t count);
  template <typename T> T* upload(const T* host, size_t count);
  R* upload_conv(const double* host, size_t count);
  void dfree(void* p);
  void zero(void* p, size_t bytes);
  void realloc_partials();
  void upload_items();
  void sync_desc();
  void invalidate_graphs();
  void launch_iterations(int mode, int count);
  hipGraphExec_t chain_graph(int mode, int count);   // the captured chain of `count` iterations
  void upload_chunks();                              // the geometry's runs, chunks and slots
  void build_operator_items();
  void build_prior_items();
  void prime(int mode);       // Algorithm 3: the data gradient and Psi A of the current state
  void adaptive_buffers();
  void forward(int src_img, int mode, int out_vis);
  void adjoint(int src_vis, int use_cfac, int dst_img);
  void finalize(int q, int count, int scalar);
  void read_scalars(double* out);
  void write_scalar(int idx, double v);
  void put_img(int slot, const double* src, int comps);
  void put_coef(int slot, const double* src);
  void get_coef(int slot, double* dst);
  void put_vis(int slot, const double* src);
  void get_vis(int slot, double* dst, double scale);
  LaunchArgs la(const DevItems& d, hipStream_t s = nullptr) const;

  Geometry geo_;
  hipStream_t s0_ = nullptr, s1_ = nullptr;
  hipEvent_t ev_fork_ = nullptr, ev_join_ = nullptr;
  int* d_perm_ = nullptr;        // the row permutation on the device (set_data_dev), made on first use
  int* d_flag_ = nullptr;        // set_data_dev's non-finite flag
  int* d_active_ = nullptr;      // adaptive runs: problems still running (device) ...
  int* h_active_ = nullptr;      // ... and its pinned host copies, one per chunk parity
  hipEvent_t ev_active_[2] = {nullptr, nullptr};
  ProbDesc h_;
  ProbDesc* d_desc_ = nullptr;
  bool desc_dirty_ = true;
  ItemSet items_;
  DevItems d_img_, d_rows_, d_cols_, d_p6_, d_p7_, d_p7f_, d_dirac_, d_synfinal_, d_synsplit_, d_coarse_;
  int c_level_ = 1 << 20;     // first level handled by the fused coarse kernel (> levels: none)
  DevItems d_ana_[kMaxLevels + 1], d_syn_[kMaxLevels + 1];
  DevItems d_ana_d_[kMaxLevels + 1], d_syn_d_[kMaxLevels + 1];
  PassLists pl_;
  int cells_ = 512;     // FFT cells per workgroup of the column passes
  int rcells_ = 2048;   // ... and of the row passes (several image rows per workgroup)
  Tuning tuning_;
  int gen_parts_ = 1, ana_parts_ = 0;
  size_t coef_elems_ = 0;
  size_t bytes_ = 0;
  std::vector<void*> allocs_;
  std::map<uint64_t, hipGraphExec_t> graphs_;
};

// Several solves advanced together: one launch per pass covers every member (their work lists
// concatenated, each item naming its member's descriptor), so small problems fill the GPU
// together and the launch latency is paid once per batch.  Members keep their own device state;
// they must share the precision R and the tap count, and every member needs a wavelet prior for
// the modes with the sparsity term.  Not re-entrant; the members must not run meanwhile.
template <typename R>
struct Batch {
  Batch(const std::vector<Engine<R>*>& members, hipStream_t stream);
  ~Batch();
  Batch(const Batch&) = delete;
  Batch& operator=(const Batch&) = delete;
  void run(int mode, int iters);       // graph replay; returns with the work queued on stream()
  void capture(int mode);              // capture the graphs run() replays (no work is launched)
  void profile(int mode, int iters, double* ms);   // per-pass times over all members (as Engine)
  // adaptive stopping per member (as Engine::run_adaptive); iters_out: iterations per member
  void run_adaptive(int mode, int max_iters, int check_every, const double* stop, int* iters_out);
  // the pieces of an adaptive run for a caller that polls on its own: capture the chunk graph
  // (no work launched), and queue `chunks` chunks (the members' criteria set by stop_begin)
  void capture_adaptive(int mode, int check_every);
  void launch_adaptive(int mode, int chunks, int check_every);
  hipStream_t stream() const { return s0_; }
  int size() const { return (int)members_.size(); }

 private:
  hipGraphExec_t graph(int mode, int count);
  hipGraphExec_t adaptive_graph(int mode, int count);
  void adaptive_buffers();
  std::vector<Engine<R>*> members_;
  hipStream_t s0_ = nullptr, s1_ = nullptr;
  hipEvent_t ev_fork_ = nullptr, ev_join_ = nullptr;
  int* d_active_ = nullptr;
  int* h_active_ = nullptr;
  hipEvent_t ev_active_[2] = {nullptr, nullptr};
  ProbDesc* d_descs_ = nullptr;
  std::vector<void*> allocs_;
  PassLists pl_;
  std::map<uint64_t, hipGraphExec_t> graphs_;
};

}  // namespace psara
