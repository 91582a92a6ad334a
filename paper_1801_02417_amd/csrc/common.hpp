// Internal types shared by the HIP kernels and the host engine.
//
// Every kernel works on a batch of independent solves: it receives an array of
// problem descriptors (device memory) and a work list whose entry for
// blockIdx.x names the problem and the piece of it (tile, line block, chunk)
// that the workgroup processes.  A single solve is a batch of one.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psara {

constexpr int kMaxBases = 9;     // Dirac + Db1..Db8
constexpr int kMaxFilter = 16;   // Db8 has 16 taps
constexpr int kMaxTaps = 8;      // Kaiser-Bessel taps per dimension
constexpr int kMaxCheb = 17;     // Chebyshev coefficients per tap (degree <= 16)
constexpr int kMaxLevels = 8;
constexpr int kRunMax = 32;         // longest run of same-window visibilities one lane group takes
constexpr int kChunkEntries = 1024; // largest gridding chunk (entries per workgroup, staged in LDS)
constexpr int kGridThreads = 512;   // threads per gridding workgroup (64 lane groups of 8)
constexpr int kSmallChunk = 16;     // a chunk of at most this many entries is gridded by one wave
constexpr int kGridFactorItem = -1;  // gridding work item that stores the pass's factor
constexpr int kGridSmallItem = -2;   // gridding work item of up to eight small chunks, one per wave
constexpr int kBatchChunk = 8;       // iterations per captured graph of a batch
constexpr int kChain = 32;           // iterations per captured chain of a single solve
constexpr int kMaxDegridTile = 32;  // largest de-gridding tile side (the geometry picks 16 or 32)
// de-gridding tile side for a grid of side K: 32 from K = 64 on (a 32-cell tile stages a 39-cell
// window with T = 8, 1.49 reads per grid cell against 2.07 for 16-cell tiles), 16 below
constexpr int degrid_tile(int K) { return K >= 64 ? kMaxDegridTile : kMaxDegridTile / 2; }
constexpr int kDegridItem = 256;        // default visibilities per de-gridding work item
constexpr int kGridTile = 16;       // side of the gridding tiles (the de-gridding tiles are P.ts)
// analysis tiling (the analysis_wide tuning, a problem's ana_wide), two bits: kAnaWide, 16-wide
// output tiles for FP32 bands of side >= 128 (else 8-wide); kAnaAllBases, level-1 items of the
// iterations that run every basis over one staged image region (kAllBases in the item's basis
// field) instead of one item per basis
constexpr int kAnaWide = 1;
constexpr int kAnaAllBases = 2;
constexpr int kAllBases = -1;

// Chebyshev degree of the per-tap Kaiser-Bessel expansions (max error ~1e-10 / ~1e-15)
// SARA tile sides: analysis output tile per band for an input of side 2h, and synthesis
// output tile for an output of side m (smaller tiles give more workgroups at coarse levels)
template <typename R> __host__ __device__ constexpr int dwt_ana_tile(int h, bool wide = true) {
  return (sizeof(R) == 4 && wide && h >= 128) ? 16 : (h < 8 ? h : 8);
}
template <typename R> __host__ __device__ constexpr int dwt_syn_tile(int m) { return m < 16 ? m : 16; }

template <typename R> struct KbDeg { static constexpr int value = sizeof(R) == 4 ? 9 : 16; };

// image-space buffers (N pixels x 4 Stokes, or x 2 for Z / D).  The wavelet part of Psi A that
// the primal step reads is IMG_PSIA + IMG_PSIA2: the iteration's synthesis splits the bases over
// two workgroups per tile, one writing each; every other writer of IMG_PSIA zeroes IMG_PSIA2.
enum ImgSlot { IMG_S = 0, IMG_X, IMG_C, IMG_PSIA, IMG_PHIB, IMG_TMP, IMG_TMP2, IMG_PSIA2, IMG_Z, IMG_D, NUM_IMG };
// visibility-space buffers (M rows x 4 complex, sorted order)
enum VisSlot { VIS_Y = 0, VIS_BV, VIS_R, NUM_VIS };
// coefficient-space buffers (nbases * N x 4)
enum CoefSlot { COEF_A = 0, COEF_GW, COEF_TMP, NUM_COEF };
// FP64 scalar slots per problem
enum Scalar {
  SC_CFAC = 0,      // B = SC_CFAC * Bv (lazy l2-ball factor)
  SC_VNORM2,        // ||B~/rho2 - Y||^2 of the last dual-B step
  SC_GFAC,          // factor of the last gridding pass, applied when its slots are summed
  SC_RES2,          // ||Y - phi(S)||^2
  SC_DOT,           // generic reduction results
  SC_NRM2,
  SC_RV0, SC_RV1, SC_RV2, SC_RV3,      // ||X - S||^2 per Stokes
  SC_SN0, SC_SN1, SC_SN2, SC_SN3,      // ||2S - X||^2 per Stokes
  SC_RIMG2,         // sum of squares of the Stokes-I residual image
  SC_ZETA,
  SC_NPCOUNT,
  SC_OBJ,
  SC_MEAN, SC_SQ,   // coefficient moments
  // adaptive stopping (Sec. 4.6 criteria, evaluated on the device): a problem whose criteria
  // hold is halted, and every kernel then leaves its workgroups at once (0 outside such runs)
  SC_HALT,          // 1: the problem's iterations stop
  SC_ITERS,         // iterations run by the current adaptive stage
  SC_STOP_THETA,    // residual bound (1 + theta) epsilon
  SC_STOP_RV,       // bound of the largest relative variation of the four maps
  SC_STOP_NP,       // bound of N_p in percent (< 0: not used)
  SC_STOP_MAXIT,    // halt once SC_ITERS reaches it (0: no bound on the device)
  NUM_SCALARS = 32
};
static_assert(SC_STOP_MAXIT < NUM_SCALARS, "scalar slots");
// Partial sums per problem, each a (sum, compensation) pair of doubles: first the de-grid
// region (n_p6 pairs), then kGenQ generic regions of gen_stride pairs each, then one pair per
// gridding chunk for the fused de-grid + grid pass.
constexpr int kGenQ = 8;

// Per-problem descriptor.  Pointers are typed by the engine's real type R.
struct ProbDesc {
  int n, K, T, levels;
  int nbases, has_dirac, nwav, ts;      // ts = grid tile side
  int ntile_side, deg, n_p6, gen_stride;
  int ntile_side_g;       // gridding tiles per side (side kGridTile)
  int n_slots;            // gridding chunks (= partial slots) of the problem
  int dg_item;            // visibilities per de-gridding work item
  int ana_wide;           // analysis tiling: kAnaWide | kAnaAllBases bits
  long long M;
  double tau, rho1, rho2, rho3, eps, gamma, norm;   // norm = 1/sqrt(nbases)
  double delta;                                     // reweighting delta in use
  void* img[NUM_IMG];
  void* vis[NUM_VIS];
  void* coef[NUM_COEF];
  void* ll;            // DWT level scratch: per wavelet basis, levels 1..L-1
  long long ll_stride; // elements (V4) per basis in ll
  void* grid;          // K*K cells of 4 complex, transposed layout [k2][k1]
  void* half;          // K*n cells: FFT intermediate [k2][r]
  const int* vis_k0;   // packed window starts (k1 << 16 | k2), sorted order
  const void* vis_frac;   // (f1, f2) per vis, type R
  const void* mix;        // NULL (the fixed L) or per sorted vis the 4 x 4 complex L D_m^T, row-major
  int tv_kind;            // 0: the SARA prior; 1: TV; 2: l1 + TV (Algorithm 3; A = [Dirac, d1, d2] blocks)
  double tvw[4];          // TV weights per Stokes map
  double l1w[4];          // l1 weights per Stokes map (l1 + TV)
  const int* own_ptr;     // ntiles+1: sorted-vis range whose window starts in each tile
  const int* run_pack;    // gridding runs (pack_run): entry offset in the chunk, length, window start in the tile
  const int2* chunk_ent;  // list-entry range [lo, hi) of each gridding chunk
  void* gpart;            // gridding partial slots: n_slots x (kGridTile + T - 1)^2 cells, k2-major
  const int4* chunks;     // gridding chunks {tile, first run, end run, partial slot}
  const int2* tile_slots; // per gridding tile: {first partial slot, count} (count 0: no visibilities)
  const int* slot_box;    // per partial slot: the cells its chunk's windows cover (pack_box), offsets in the region
  const int* tile_box;    // per gridding tile: the union of its slots' boxes
  const int* small_ids;   // the chunks of at most kSmallChunk entries, heaviest first (eight per work item)
  const void* kbpoly;     // T x (deg+1) per-tap kernel polynomial coefficients (ascending), type R
  const void* twiddle;    // K complex exp(-2 pi i j / K), type R
  const void* deapod;     // n scaling factors 1/psi_hat((j - n/2)/K), type R
  const void* filters;    // nwav x 16 low-pass filters (zero padded), type R
  int wav_len[8];         // filter length of each wavelet basis
  double* partials;       // [n_p6 pairs][kGenQ x gen_stride pairs][n_slots pairs]
  double* scal;           // NUM_SCALARS
  long long ll_off[kMaxLevels + 1];  // element offset of level l's LL inside a basis block
};

// The cells a gridding chunk's windows cover inside its (kGridTile + T - 1)^2 region: k1 offsets
// [lo1, hi1] and k2 offsets [lo2, hi2], one byte each.  The gridding writes only these cells of
// its slot (the others hold zero), and the column inverse FFT skips a tile's slots at cells
// outside the union of their boxes.
__host__ __device__ constexpr int pack_box(int lo1, int hi1, int lo2, int hi2) {
  return lo1 | (hi1 << 8) | (lo2 << 16) | (hi2 << 24);
}
__host__ __device__ inline bool in_box(int box, int o1, int o2) {
  return o1 >= (box & 255) && o1 <= ((box >> 8) & 255) && o2 >= ((box >> 16) & 255) && o2 <= ((box >> 24) & 255);
}

// log2 of a power of two
__host__ __device__ inline int lg2(int p) { return __builtin_ctz((unsigned)p); }
// q / d for 0 <= q < 2^14 and 1 <= d <= 128 by a float multiply: (q + 0.5) times the rounded
// reciprocal of d (even one ulp off) stays inside [floor(q / d), floor(q / d) + 1), which holds
// for every such q and d; rcp = 1 / d is computed once.
__device__ inline int small_div(int q, float rcp) { return (int)(((float)q + 0.5f) * rcp); }

// dst[q] = load(q) for q < n <= U * blockDim.x, each thread taking q = threadIdx.x + u * blockDim.x:
// every load of the thread is issued before its first LDS store, so the loads are in flight
// together (a loop that stores each element as it arrives waits for one load at a time).
template <int U, class T, class Load>
__device__ inline void stage_lds(T* dst, int n, Load&& load) {
  T v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int q = threadIdx.x + u * blockDim.x;
    if (q < n) v[u] = load(q);
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int q = threadIdx.x + u * blockDim.x;
    if (q < n) dst[q] = v[u];
  }
}

// A gridding run in one word: the offset of its first entry in its chunk (< 1024), its length
// (1 .. 32) and its window start relative to its tile (o1, o2 < 16).
__host__ __device__ constexpr int pack_run(int off, int len, int o1, int o2) {
  return off | ((len - 1) << 10) | (o1 << 15) | (o2 << 19);
}
static_assert(kChunkEntries <= 1024 && kRunMax <= 32 && kGridTile <= 16, "run fields");

// --------------------------------------------------------------------------------------------
// small vector types
template <typename R> struct alignas(4 * sizeof(R)) V4 { R x, y, z, w; };
template <typename R> struct alignas(2 * sizeof(R)) V2 { R x, y; };
template <typename R> struct cplx { R re, im; };
// one grid cell: the four Stokes channels, complex (32 B in FP32, 64 B in FP64)
template <typename R> struct alignas(16) Cell { cplx<R> s[4]; };

template <typename R> __host__ __device__ inline cplx<R> cmk(R a, R b) { cplx<R> c; c.re = a; c.im = b; return c; }
template <typename R> __host__ __device__ inline cplx<R> cadd(cplx<R> a, cplx<R> b) { return cmk(a.re + b.re, a.im + b.im); }
template <typename R> __host__ __device__ inline cplx<R> csub(cplx<R> a, cplx<R> b) { return cmk(a.re - b.re, a.im - b.im); }
template <typename R> __host__ __device__ inline cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return cmk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename R> __host__ __device__ inline cplx<R> cscale(cplx<R> a, R s) { return cmk(a.re * s, a.im * s); }
template <typename R> __host__ __device__ inline cplx<R> cmuli(cplx<R> a) { return cmk(-a.im, a.re); }   // i * a
template <typename R> __host__ __device__ inline cplx<R> cconj(cplx<R> a) { return cmk(a.re, -a.im); }

// --------------------------------------------------------------------------------------------
// compensated FP64 sums (Neumaier), combinable in a fixed tree
struct KSum {
  double s, c;
  __host__ __device__ KSum() : s(0.0), c(0.0) {}
  __host__ __device__ void add(double v) {
    double t = s + v;
    if (fabs(s) >= fabs(v)) c += (s - t) + v; else c += (v - t) + s;
    s = t;
  }
  __host__ __device__ void merge(const KSum& o) { add(o.s); c += o.c; }
  __host__ __device__ double value() const { return s + c; }
};

__device__ inline KSum wave_reduce(KSum k) {
  for (int off = 32; off > 0; off >>= 1) {
    KSum o;
    o.s = __shfl_xor(k.s, off, 64);
    o.c = __shfl_xor(k.c, off, 64);
    k.merge(o);
  }
  return k;
}

// Block-wide deterministic reduction; every thread returns the same total.
// `scratch` must hold 2 * (blockDim.x / 64) doubles of shared memory.
__device__ inline KSum block_reduce(KSum k, double* scratch) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  k = wave_reduce(k);
  __syncthreads();
  if (lane == 0) { scratch[2 * wave] = k.s; scratch[2 * wave + 1] = k.c; }
  __syncthreads();
  KSum t;
  for (int w = 0; w < nw; ++w) { KSum o; o.s = scratch[2 * w]; o.c = scratch[2 * w + 1]; t.merge(o); }
  __syncthreads();
  return t;
}

// true when an adaptive run has stopped this problem (its kernels then do nothing)
__device__ inline bool halted(const ProbDesc& P) { return P.scal[SC_HALT] != 0.0; }

// the partial pairs of the fused de-grid + grid pass, one per gridding chunk (n_slots pairs
// after the generic regions)
__host__ __device__ inline double* chunk_partials(const ProbDesc& P) {
  return P.partials + 2 * ((size_t)P.n_p6 + (size_t)kGenQ * P.gen_stride);
}

// Sum `count` (s, c) pairs from `parts` in a fixed order with the whole block.
__device__ inline double block_sum_partials(const double* parts, int count, double* scratch) {
  KSum k;
  for (int i = threadIdx.x; i < count; i += blockDim.x) {
    KSum o; o.s = parts[2 * i]; o.c = parts[2 * i + 1]; k.merge(o);
  }
  return block_reduce(k, scratch).value();
}

// --------------------------------------------------------------------------------------------
// Kaiser-Bessel weights: the T weights psi(f - i), i = 0..T-1, of one dimension.  With the
// window start k0 = ceil(t - T/2) the fractional offset f = t - k0 lies in (T/2 - 1, T/2], so
// every tap's argument spans one unit interval and u = 2f - T + 1 in (-1, 1] is common to all
// taps.  Each tap carries its own polynomial in u on that interval (Horner's rule).
template <typename R, int T>
__device__ inline R kb_tap(R u, const R* __restrict__ c) {
  constexpr int DEG = KbDeg<R>::value;
  R acc = c[DEG];
#pragma unroll
  for (int k = DEG - 1; k >= 0; --k) acc = acc * u + c[k];
  return acc;
}

template <typename R, int T>
__device__ inline void kb_weights(R f, const R* __restrict__ poly, R* w) {
  constexpr int DEG = KbDeg<R>::value;
  const R u = R(2) * f - R(T - 1);
#pragma unroll
  for (int i = 0; i < T; ++i) w[i] = kb_tap<R, T>(u, poly + i * (DEG + 1));
}

}  // namespace psara
