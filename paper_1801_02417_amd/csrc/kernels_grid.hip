// Interpolation matrix G of the measurement operator and its adjoint (Sec. 4.1, eq.
// meas_op), fused with the Stokes-to-brightness mixing L (Sec. 2.1) and the dual update
// of the data-fidelity term (Algorithm 1, l2-ball steps; radius epsilon, see the
// data-fidelity paragraph of Sec. 3.3.2).
//
// Visibilities are sorted once (at set-up) by the grid tile that holds their window start
// k0 = ceil(t - T/2).  De-gridding stages a tile plus its (T-1)-cell halo of the grid in LDS
// and lets one thread per visibility gather its T x T taps from there.  Gridding is done by
// the owner of each visibility's window start: the workgroups of a tile accumulate the taps of
// its visibilities over the tile plus halo in LDS and write that region to a partial slot of
// their own with plain stores; the column inverse FFT sums the slots covering each cell in a
// fixed order, so no global atomics are used.  Both also exist as one fused pass over the
// gridding chunks (a chunk's taps all lie in the region it accumulates), which the iterations
// use when no other branch runs beside them.
//
// The dual variable B is kept as B = c * Bv: the de-gridding pass writes
// Bv = B/rho2 + phi(X) - Y and the FP64 partial sums of ||Bv||^2; the gridding pass reduces
// those partials (fixed order, compensated) to c = rho2 * max(0, 1 - epsilon/||Bv||), which
// both it and the next iteration's de-gridding apply on the fly.  This equals
// B~ - rho2 P_B(Y,eps)(B~/rho2) without a second pass over the visibilities.
#include <mutex>
#include <set>
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"

namespace psara {

// ---------------------------------------------------------------------------------------------
// Pieces shared by the de-grid, grid and fused passes (one definition, so that the fused pass
// computes exactly what the separate ones do).

// v_s = sum_j w2[j] sum_i w1[i] win[(r2 + j) * ws + r1 + i].s: the T x T taps of a window held
// in LDS as k2-major rows of ws cells
template <typename R, int T>
__device__ inline void interpolate(const Cell<R>* win, int ws, int r1, int r2, const R* w1, const R* w2,
                                   cplx<R> v[4]) {
#pragma unroll
  for (int s = 0; s < 4; ++s) v[s] = cmk(R(0), R(0));
#pragma unroll
  for (int j = 0; j < T; ++j) {
    const Cell<R>* row = win + (r2 + j) * ws + r1;
    cplx<R> t[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) t[s] = cmk(R(0), R(0));
#pragma unroll
    for (int i = 0; i < T; ++i) {
      const Cell<R> c = row[i];
#pragma unroll
      for (int s = 0; s < 4; ++s) { t[s].re += w1[i] * c.s[s].re; t[s].im += w1[i] * c.s[s].im; }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) { v[s].re += w2[j] * t[s].re; v[s].im += w2[j] * t[s].im; }
  }
}

// the brightness products of row m from its de-gridded Stokes values: [I+Q, U+iV, U-iV, I-Q],
// or with known Mueller matrices the row times L D_m^T
template <typename R>
__device__ inline Cell<R> brightness(const ProbDesc& P, int m, const cplx<R> v[4]) {
  Cell<R> phi;
  if (P.mix) {
    const cplx<R>* __restrict__ mx = (const cplx<R>*)P.mix + (size_t)m * 16;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      cplx<R> a = cmul(v[0], mx[j]);
#pragma unroll
      for (int s = 1; s < 4; ++s) a = cadd(a, cmul(v[s], mx[4 * s + j]));
      phi.s[j] = a;
    }
  } else {
    phi.s[0] = cadd(v[0], v[1]);
    phi.s[1] = cadd(v[2], cmuli(v[3]));
    phi.s[2] = csub(v[2], cmuli(v[3]));
    phi.s[3] = csub(v[0], v[1]);
  }
  return phi;
}

// What the de-grid pass's row m reads besides its window: Y, and for DG_DUAL the previous Bv.
template <typename R>
struct RowIn {
  Cell<R> y, bv;
};
template <typename R, int MODE>
__device__ inline RowIn<R> row_inputs(const ProbDesc& P, long long m, int src_slot) {
  RowIn<R> r{};
  if (MODE != DG_FORWARD) r.y = ((const Cell<R>*)P.vis[VIS_Y])[m];
  if (MODE == DG_DUAL) r.bv = ((const Cell<R>*)P.vis[src_slot])[m];
  return r;
}

// The de-grid pass's row m for MODE (not DG_FORWARD) from its de-gridded Stokes values and its
// inputs, with the squared moduli of its eight reals added to acc.  DG_DUAL: Bv = cb Bv_old +
// phi - Y (cb = c/rho2); DG_RESIDUAL: Y - phi; DG_STOKES: per Stokes map Phi S - Y L^{-1}
// (I = (Y1 + Y4) / 2, Q = (Y1 - Y4) / 2, U = (Y2 + Y3) / 2, V = -i (Y2 - Y3) / 2).
template <typename R, int MODE>
__device__ inline Cell<R> degrid_row_in(const ProbDesc& P, int m, const cplx<R> v[4], const RowIn<R>& in, R cb,
                                        KSum& acc) {
  const Cell<R>& y = in.y;
  Cell<R> o;
  if (MODE == DG_STOKES) {
    const R h = R(0.5);
    o.s[0] = csub(v[0], cscale(cadd(y.s[0], y.s[3]), h));
    o.s[1] = csub(v[1], cscale(csub(y.s[0], y.s[3]), h));
    o.s[2] = csub(v[2], cscale(cadd(y.s[1], y.s[2]), h));
    const cplx<R> dv = csub(y.s[1], y.s[2]);
    o.s[3] = csub(v[3], cmk(h * dv.im, -h * dv.re));
  } else {
    const Cell<R> phi = brightness<R>(P, m, v);
    if (MODE == DG_DUAL) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        o.s[s].re = cb * in.bv.s[s].re + phi.s[s].re - y.s[s].re;
        o.s[s].im = cb * in.bv.s[s].im + phi.s[s].im - y.s[s].im;
      }
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s) o.s[s] = csub(y.s[s], phi.s[s]);
    }
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const double re = (double)o.s[s].re, im = (double)o.s[s].im;
    acc.add(re * re);
    acc.add(im * im);
  }
  return o;
}

template <typename R, int MODE>
__device__ inline R dual_factor(const ProbDesc& P) {
  return MODE == DG_DUAL ? R(P.scal[SC_CFAC] / P.rho2) : R(0);
}

template <typename R, int MODE>
__device__ inline Cell<R> degrid_row(const ProbDesc& P, int m, const cplx<R> v[4], int src_slot, KSum& acc) {
  return degrid_row_in<R, MODE>(P, m, v, row_inputs<R, MODE>(P, m, src_slot), dual_factor<R, MODE>(P), acc);
}

// The gridded channels of row m with value b: B L^H (I = B1 + B4, Q = B1 - B4, U = B2 + B3,
// V = i (B3 - B2)); with known Mueller matrices B (L D_m^T)^H; GR_STOKES: the row itself (it is
// per Stokes map already).  Returns the largest magnitude among the eight reals.
template <typename R, int MODE>
__device__ inline R grid_channels(const ProbDesc& P, int m, const Cell<R>& b, V4<R>& u0, V4<R>& u1) {
  if (MODE == GR_STOKES) {
    u0.x = b.s[0].re; u0.y = b.s[0].im; u0.z = b.s[1].re; u0.w = b.s[1].im;
    u1.x = b.s[2].re; u1.y = b.s[2].im; u1.z = b.s[3].re; u1.w = b.s[3].im;
  } else if (P.mix) {
    const cplx<R>* __restrict__ mx = (const cplx<R>*)P.mix + (size_t)m * 16;
    cplx<R> u[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      cplx<R> a = cmul(b.s[0], cconj(mx[4 * s]));
#pragma unroll
      for (int j = 1; j < 4; ++j) a = cadd(a, cmul(b.s[j], cconj(mx[4 * s + j])));
      u[s] = a;
    }
    u0.x = u[0].re; u0.y = u[0].im; u0.z = u[1].re; u0.w = u[1].im;
    u1.x = u[2].re; u1.y = u[2].im; u1.z = u[3].re; u1.w = u[3].im;
  } else {
    u0.x = (b.s[0].re + b.s[3].re); u0.y = (b.s[0].im + b.s[3].im);
    u0.z = (b.s[0].re - b.s[3].re); u0.w = (b.s[0].im - b.s[3].im);
    u1.x = (b.s[1].re + b.s[2].re); u1.y = (b.s[1].im + b.s[2].im);
    u1.z = -(b.s[2].im - b.s[1].im); u1.w = (b.s[2].re - b.s[1].re);
  }
  return fmax(fmax(fmax(fabs(u0.x), fabs(u0.y)), fmax(fabs(u0.z), fabs(u0.w))),
              fmax(fmax(fabs(u1.x), fabs(u1.y)), fmax(fabs(u1.z), fabs(u1.w))));
}

// ---------------------------------------------------------------------------------------------
// One row of the de-grid pass: its window (starting at region offsets (pk >> 16) - c1,
// (pk & 0xffff) - c2 of the staged band, ws cells wide) interpolated with its taps, then stored.
template <typename R, int MODE, int T>
__device__ __forceinline__ void degrid_one(const ProbDesc& P, const Cell<R>* win, int ws, int c1, int c2, int m, int pk,
                                           V2<R> f, const RowIn<R>& in, R cb, Cell<R>* __restrict__ out, KSum& acc) {
  R w1[T], w2[T];
  kb_weights<R, T>(f.x, (const R*)P.kbpoly, w1);
  kb_weights<R, T>(f.y, (const R*)P.kbpoly, w2);
  cplx<R> v[4];
  interpolate<R, T>(win, ws, (pk >> 16) - c1, (pk & 0xffff) - c2, w1, w2, v);
  if (MODE == DG_FORWARD) out[m] = brightness<R>(P, m, v);
  else out[m] = degrid_row_in<R, MODE>(P, m, v, in, cb, acc);
}

// window elements a de-grid thread stages: the largest window ((ts + T - 1)^2 cells, ts <= 32)
// over the 256 threads of a workgroup
template <int T> constexpr int kDegridWin = ((kMaxDegridTile + T - 1) * (kMaxDegridTile + T - 1) + 255) / 256;

// P6: de-grid + L mixing (+ dual B).  items: {prob, tile | rows << 16, first sorted vis, partial
// index | lo << 20 | hi << 25}; an item holds P.dg_item rows of the tile (fewer at its end), a
// thread takes every blockDim.x-th; lo and hi are the smallest and largest window start k1 of
// its rows relative to the tile, so the k1 band [lo, hi + T - 1] of the tile window is all the
// item stages
template <typename R, int MODE, int T>
__global__ void __launch_bounds__(256)
degrid_kernel(const ProbDesc* __restrict__ descs, const int4* __restrict__ items, int src_slot, int out_slot) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Cell<R>* win = (Cell<R>*)smem_raw;
  __shared__ double red[8];
  const int4 it = items[blockIdx.x];
  const ProbDesc& P = descs[it.x];
  const int K = P.K, ts = P.ts, nts = P.ntile_side;
  const int tile = it.y & 0xffff, vend = it.z + (it.y >> 16);
  const int t1 = tile / nts, t2 = tile - t1 * nts;
  const int W = ts + T - 1;
  const Cell<R>* __restrict__ grid = (const Cell<R>*)P.grid;
  const int b1 = t1 * ts, b2 = t2 * ts;
  Cell<R>* __restrict__ out = (Cell<R>*)P.vis[out_slot];
  const R cb = dual_factor<R, MODE>(P);
  const int mf = it.z + threadIdx.x;
  const int part = it.w & 0xfffff, lo = (it.w >> 20) & 31, Wb = ((it.w >> 25) & 31) - lo + T;
  KSum acc;
  if constexpr (sizeof(R) == 4) {
    // FP32: the thread's first row and what it reads are requested before the halt test and
    // the window, so those loads are in flight together; lo and hi come from the threads
    // holding the first and the last row
    int pk0 = 0;
    V2<R> f0{};
    RowIn<R> in0{};
    if (mf < vend) {
      pk0 = P.vis_k0[mf];
      f0 = ((const V2<R>*)P.vis_frac)[mf];
      in0 = row_inputs<R, MODE>(P, mf, src_slot);
    }
    if (halted(P)) return;                 // stopped by an adaptive run
    const float rwb = 1.0f / (float)Wb;
    stage_lds<kDegridWin<T>>(win, W * Wb, [&](int q) {
      const int a = small_div(q, rwb), b = q - a * Wb;          // a: k2 offset, b: k1 offset - lo
      return grid[(size_t)((b2 + a) & (K - 1)) * K + ((b1 + lo + b) & (K - 1))];
    });
    __syncthreads();
    // the first row from the values loaded above, later rows (items longer than the
    // workgroup) loaded as they come
    if (mf < vend) degrid_one<R, MODE, T>(P, win, Wb, b1 + lo, b2, mf, pk0, f0, in0, cb, out, acc);
    for (int m = mf + blockDim.x; m < vend; m += blockDim.x)
      degrid_one<R, MODE, T>(P, win, Wb, b1 + lo, b2, m, P.vis_k0[m], ((const V2<R>*)P.vis_frac)[m],
                             row_inputs<R, MODE>(P, m, src_slot), cb, out, acc);
  } else {
    // FP64 (the interpolation takes every register): rows are read as they are de-gridded
    if (halted(P)) return;                 // stopped by an adaptive run
    const float rwb = 1.0f / (float)Wb;
    stage_lds<kDegridWin<T>>(win, W * Wb, [&](int q) {
      const int a = small_div(q, rwb), b = q - a * Wb;
      return grid[(size_t)((b2 + a) & (K - 1)) * K + ((b1 + lo + b) & (K - 1))];
    });
    __syncthreads();
    for (int m = mf; m < vend; m += blockDim.x) {
      const int pk = P.vis_k0[m];
      const V2<R> f = ((const V2<R>*)P.vis_frac)[m];
      R w1[T], w2[T];
      kb_weights<R, T>(f.x, (const R*)P.kbpoly, w1);
      kb_weights<R, T>(f.y, (const R*)P.kbpoly, w2);
      cplx<R> v[4];
      interpolate<R, T>(win, Wb, (pk >> 16) - b1 - lo, (pk & 0xffff) - b2, w1, w2, v);
      if (MODE == DG_FORWARD) out[m] = brightness<R>(P, m, v);
      else out[m] = degrid_row<R, MODE>(P, m, v, src_slot, acc);
    }
  }
  if (MODE != DG_FORWARD) {
    const KSum tot = block_reduce(acc, red);
    if (threadIdx.x == 0) {
      P.partials[2 * part] = tot.s;
      P.partials[2 * part + 1] = tot.c;
    }
  }
}

template <typename R, int T>
void launch_degrid_t(int mode, const LaunchArgs& a, size_t shm, int src_slot, int out_slot) {
  const dim3 grid(a.nitems), block(256);
  if (mode == DG_DUAL) {
    hipLaunchKernelGGL((degrid_kernel<R, DG_DUAL, T>), grid, block, shm, a.stream, a.descs, a.items, src_slot, out_slot);
  } else if (mode == DG_STOKES) {
    hipLaunchKernelGGL((degrid_kernel<R, DG_STOKES, T>), grid, block, shm, a.stream, a.descs, a.items, src_slot, out_slot);
  } else if (mode == DG_FORWARD) {
    hipLaunchKernelGGL((degrid_kernel<R, DG_FORWARD, T>), grid, block, shm, a.stream, a.descs, a.items, src_slot, out_slot);
  } else {
    hipLaunchKernelGGL((degrid_kernel<R, DG_RESIDUAL, T>), grid, block, shm, a.stream, a.descs, a.items, src_slot, out_slot);
  }
}

// taps: the kernel support T of every problem in the launch (4, 6 or 8)
template <typename R>
void launch_degrid(int mode, const LaunchArgs& a, int max_ts, int taps, int src_slot, int out_slot) {
  if (a.nitems <= 0) return;
  const int W = max_ts + taps - 1;
  const size_t shm = (size_t)W * W * sizeof(Cell<R>);
  if (taps == 4) launch_degrid_t<R, 4>(mode, a, shm, src_slot, out_slot);
  else if (taps == 6) launch_degrid_t<R, 6>(mode, a, shm, src_slot, out_slot);
  else launch_degrid_t<R, 8>(mode, a, shm, src_slot, out_slot);
}

// ---------------------------------------------------------------------------------------------
// P7: grid (adjoint of G, after mixing by L^H).  items: {prob, chunk, first row, end row}
// for a chunk of more than kSmallChunk entries, {prob, kGridFactorItem, -, -} for the factor
// item, {prob, kGridSmallItem, first of small_ids, count} for up to eight small chunks
// (grid_small above: one wave each, summed in registers in a fixed order).
//
// The grid is cut into kGridTile x kGridTile tiles and every visibility belongs to the tile
// holding its window start, so it is gridded exactly once; the workgroup accumulates the tile
// plus its (T-1)-wide halo on the high sides, (kGridTile + T - 1)^2 cells, which every window
// starting in the tile stays inside.  A tile's rows are contiguous (rows are sorted by
// de-gridding tile, then gridding tile, then window start); a chunk is a set of runs of them,
// a run being visibilities with the same window start, so all their T x T taps land on the
// same cells.  The chunk's entries (offsets and L^H-mixed values) are first staged in LDS by
// the whole workgroup.  A group of 8 lanes then takes one run: lane i owns tap row i and
// accumulates, over the run, the 8 cells of that row for the 8 real channels in registers
// (the column weights are shared through DPP lane moves), and adds the row to the tile once.
//
// The tile accumulates in 64-bit fixed point with integer LDS atomics: integer addition is
// associative, so the result does not depend on the order in which lanes arrive (the
// gridding is bitwise reproducible), and integer LDS atomics run far faster than floating
// ones.  The scale is the power of two 2^E <= 2^48 (FP32) or 2^61 (FP64) divided by
// sum_v max_c |u_v,c| over the chunk, a bound on any partial sum of a cell (the kernel weights
// are at most 1), so no sum leaves the range of the conversion; the absolute rounding per
// addition is at most 2^-49 (2^-62) of that bound.
//
// The cells of the chunk's box (those its windows reach) go to the chunk's partial slot; the
// column inverse FFT sums, for each cell, the slots of its own tile and of the up to three
// tiles whose halos cover it, in a fixed order, and multiplies the sum by the scalar factor of
// B, which the gridding leaves out: one item per problem (kGridFactorItem, first in the work
// list, so it runs beside the chunks)
// stores that factor -- GR_DUAL: c, reduced in a fixed order from the de-grid partials and
// also kept for the next iteration; GR_PLAIN: 1, or the stored c when use_cfac is set;
// GR_STOKES: 1.
//
// Fixed-point terms of the LDS accumulation: conv(a, fx) is the term of a * fx (fx a power of
// two, so a * fx is exact), value(sum) the nearest-integer sum of the terms it received.
// FP32 data: the term is the bit pattern of the double 1.5 * 2^52 + a * fx, whose mantissa holds
// rint(a * fx) (|a * fx| < 2^51) -- one conversion and one fused multiply-add.  That pattern is
// the integer 0x867 * 2^51 + rint(a * fx), so the 64-bit sum of any number of terms equals the
// sum of the roundings modulo 2^51, and with |sum| < 2^50 (the scale keeps it below 2^48 times
// the largest tap product, which is at most 1) sign-extending its low 51 bits recovers it
// exactly, whatever the order of the additions.  FP64 data use the exact conversion and a range
// of 2^61.
template <typename R> struct Fixed;
template <> struct Fixed<float> {
  static constexpr int kRange = 48;
  __device__ static unsigned long long conv(float a, double fx) {
    constexpr double kMagic = 6755399441055744.0;          // 1.5 * 2^52
    return (unsigned long long)__double_as_longlong(__fma_rn((double)a, fx, kMagic));
  }
  __device__ static long long value(unsigned long long sum) { return (long long)(sum << 13) >> 13; }
};
template <> struct Fixed<double> {
  static constexpr int kRange = 61;
  __device__ static unsigned long long conv(double a, double fx) { return (unsigned long long)__double2ll_rn(a * fx); }
  __device__ static long long value(unsigned long long sum) { return (long long)sum; }
};

// The exponent E of the chunk's fixed-point scale 2^E, with 2^E * total <= 2^kRange (total: the
// sum over the chunk's rows of their largest channel magnitude); multiplying by 2^E is exact.
template <typename R>
__device__ inline int fixed_exponent(double total) {
  return total > 0.0 ? min(Fixed<R>::kRange - (int)ceil(log2(total * (1.0 + 1e-6))), 100) : 0;
}

// What a gridding workgroup loads before its entries are staged (so those loads overlap the
// staging's): its group's first run, the chunk's box and, with POLY, this lane's tap polynomial
// (the kernels with more registers live during the staging -- the FP64 one and the fused
// de-grid + grid -- load it after the staging instead, which keeps them free of spills).
template <typename R>
struct ChunkPre {
  R cr[KbDeg<R>::value + 1];
  int run = 0;                                     // the group's first run (pack_run), 0 if none
  int box = 0;
};

template <typename R, int T>
__device__ inline void load_poly(const ProbDesc& P, R* cr) {
  constexpr int DEG = KbDeg<R>::value;
  const int lane8 = threadIdx.x & 7;
  const R* __restrict__ poly = (const R*)P.kbpoly + (lane8 < T ? lane8 : 0) * (DEG + 1);
#pragma unroll
  for (int k = 0; k <= DEG; ++k) cr[k] = lane8 < T ? poly[k] : R(0);
}

template <typename R, int T, bool POLY>
__device__ inline void chunk_preload(const ProbDesc& P, const int4 ch, ChunkPre<R>& pre) {
  if (POLY) load_poly<R, T>(P, pre.cr);
  const int rr = ch.y + (threadIdx.x >> 3);
  if (rr < ch.z) pre.run = P.run_pack[rr];
  pre.box = P.slot_box[ch.w];
}

// Lane moves inside a lane group of eight with DPP (a VALU operand modifier, so no trip
// through the LDS unit): quad_bcast<K> gives every lane the value of lane K of its quad,
// half_mirror the value of lane 7 - i of its group of eight.  A double moves as two words.
template <int CTRL, typename V>
__device__ inline V dpp_move(V v) {
  static_assert(sizeof(V) % 4 == 0, "32-bit words");
  union { V v; int w[sizeof(V) / 4]; } a, b;
  a.v = v;
#pragma unroll
  for (int k = 0; k < (int)(sizeof(V) / 4); ++k) b.w[k] = __builtin_amdgcn_mov_dpp(a.w[k], CTRL, 0xf, 0xf, true);
  return b.v;
}
template <int K, typename V> __device__ inline V quad_bcast(V v) { return dpp_move<K * 0x55>(v); }
template <typename V> __device__ inline V half_mirror(V v) { return dpp_move<0x141>(v); }

// The tap product w1 * w2[j] of the lane's tap row and the group's tap column held in
// accumulator column jj.  For T = 8 the accumulator columns of the upper quad (lanes 4..7) are
// the tap columns jj ^ 4 (tap_col below): a lane then takes columns 0..3 of its own quad by a
// quad broadcast of w2 and the other four from the mirrored w2 (lane 7 - i), so every
// broadcast index is the same in both quads.  T = 4 uses the lower quad alone; T = 6 moves
// the values with a lane shuffle.
template <typename R, int T, int JJ>
__device__ inline R tap_product(R w1, R w2, R w2m) {
  if constexpr (T == 8) {
    if constexpr (JJ < 4) return w1 * quad_bcast<JJ>(w2);
    else return w1 * quad_bcast<7 - JJ>(w2m);
  } else if constexpr (T == 4) {
    return w1 * quad_bcast<JJ>(w2);
  } else {
    return w1 * __shfl(w2, JJ, 8);
  }
}
template <int T>
__device__ inline int tap_col(int jj, int lane8) { return T == 8 ? (jj ^ (lane8 & 4)) : jj; }

// f(std::integral_constant<int, J>) for J = B .. E-1, in order
template <int B, int E, class F>
__device__ inline void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Accumulates a chunk whose rows are staged in LDS (sf: fractional offsets, su: two V4 of
// gridded channels per entry, entry q the chunk's q-th row) into acc, which must be zero,
// and writes the cells of the chunk's box to its partial slot (the slot's other cells are zero
// from the allocation on and stay so).  Called by the whole workgroup.
template <typename R, int T, bool POLY>
__device__ inline void grid_chunk(const ProbDesc& P, const int4 ch,
                                  const V2<R>* sf, const V4<R>* su, unsigned long long* acc, int E,
                                  const ChunkPre<R>& pre) {
  constexpr int RG = kGridTile + T - 1;
  constexpr int DEG = KbDeg<R>::value;
  R cr[DEG + 1];                                   // this lane's tap polynomial
  if (POLY) {
#pragma unroll
    for (int k = 0; k <= DEG; ++k) cr[k] = pre.cr[k];
  } else {
    load_poly<R, T>(P, cr);
  }
  const double fx = ldexp(1.0, E);
  const int lane8 = threadIdx.x & 7;               // tap row owned by this lane
  const int grp = threadIdx.x >> 3, ngrp = blockDim.x >> 3;
  // FP64 accumulates a run's eight channels in two passes of four (T x 8 doubles would not stay
  // in registers); each channel's sum is the same either way
  constexpr int NC = sizeof(R) == 8 ? 4 : 8;
  int run = pre.run;
  for (int rr = ch.y + grp; rr - grp < ch.z; rr += ngrp) {
    const bool active = rr < ch.z;
    const int e0 = run & 1023;
    const int len = active ? ((run >> 10) & 31) + 1 : 0;
    const int o1 = (run >> 15) & 15, o2 = (run >> 19) & 15;   // window start in the tile
    // the group's next run, loaded while this one accumulates
    const int nr = rr + ngrp;
    if (nr < ch.z) run = P.run_pack[nr];
    // (one pass of eight channels, or in FP64 one pass per staged V4 of four)
#pragma unroll 1
    for (int c0 = 0; c0 < 8; c0 += NC) {
      R a[T][NC];
#pragma unroll
      for (int j = 0; j < T; ++j)
#pragma unroll
        for (int c = 0; c < NC; ++c) a[j][c] = R(0);
      for (int q = 0; q < len; ++q) {
        const V2<R> f = sf[e0 + q];
        // this lane's tap in each dimension: psi(f - lane8) from its polynomial
        const R w1 = kb_tap<R, T>(R(2) * f.x - R(T - 1), cr);
        const R w2 = kb_tap<R, T>(R(2) * f.y - R(T - 1), cr);
        R u[NC];
        const V4<R> v0 = su[2 * (e0 + q) + (NC == 8 ? 0 : c0 / 4)];
        u[0] = v0.x; u[1] = v0.y; u[2] = v0.z; u[3] = v0.w;
        if (NC == 8) {
          const V4<R> v1 = su[2 * (e0 + q) + 1];
          u[4 % NC] = v1.x; u[5 % NC] = v1.y; u[6 % NC] = v1.z; u[7 % NC] = v1.w;
        }
        const R w2m = half_mirror(w2);
        static_for<0, T>([&](auto jc) {
          constexpr int j = decltype(jc)::value;
          const R wj = tap_product<R, T, j>(w1, w2, w2m);
#pragma unroll
          for (int c = 0; c < NC; ++c) a[j][c] += wj * u[c];
        });
      }
      if (len > 0 && lane8 < T) {
        unsigned long long* row = acc + o1 + lane8;
#pragma unroll
        for (int j = 0; j < T; ++j) {
          unsigned long long* cell = row + (o2 + tap_col<T>(j, lane8)) * RG;
          // one tap column at a time: the empty asm (ordered with the atomics) keeps the
          // compiler from widening all the sums to 64 bits at once, which would spill
          if (NC == 8) {
            asm volatile("" : "+v"(a[j][0]), "+v"(a[j][1]), "+v"(a[j][2]), "+v"(a[j][3]),
                              "+v"(a[j][4 % NC]), "+v"(a[j][5 % NC]), "+v"(a[j][6 % NC]), "+v"(a[j][7 % NC]) :: "memory");
          } else {
            asm volatile("" : "+v"(a[j][0]), "+v"(a[j][1]), "+v"(a[j][2]), "+v"(a[j][3]) :: "memory");
          }
#pragma unroll
          for (int c = 0; c < NC; ++c) atomicAdd(cell + (c0 + c) * RG * RG, Fixed<R>::conv(a[j][c], fx));
        }
      }
    }
  }
  __syncthreads();
  Cell<R>* __restrict__ dst = (Cell<R>*)P.gpart + (size_t)ch.w * RG * RG;
  const double inv = ldexp(1.0, -E);
  for (int q = threadIdx.x; q < RG * RG; q += blockDim.x) {
    if (!in_box(pre.box, q % RG, q / RG)) continue;
    Cell<R> c;
#pragma unroll
    for (int s = 0; s < 4; ++s)
      c.s[s] = cmk(R((double)Fixed<R>::value(acc[(2 * s) * RG * RG + q]) * inv),
                   R((double)Fixed<R>::value(acc[(2 * s + 1) * RG * RG + q]) * inv));
    dst[q] = c;
  }
}

// A value of lane e (e the same in every lane), read into a scalar register.
template <typename V>
__device__ inline V lane_value(V v, int e) {
  static_assert(sizeof(V) % 4 == 0, "32-bit words");
  union { V v; int w[sizeof(V) / 4]; } a, b;
  a.v = v;
#pragma unroll
  for (int k = 0; k < (int)(sizeof(V) / 4); ++k) b.w[k] = __builtin_amdgcn_readlane(a.w[k], e);
  return b.v;
}

// P7 of the small chunks (at most kSmallChunk entries): one wave per chunk, an item holding up
// to eight of them (small_ids[it.z .. it.z + it.w)), no LDS and no atomics.  Lane e first loads
// entry e (its index, offsets, window start, gridded channels); a lane owns the cells
// q = lane + 64 k of the chunk's box and adds, entry by entry in list order, the entry's tap
// product times its channels -- a fixed order, so the sums are deterministic like the
// fixed-point sums of the larger chunks.  Lanes 0..T-1 evaluate the entry's k1 taps and lanes
// 8..8+T-1 its k2 taps; a cell takes the two it needs by a lane shuffle.
template <typename R, int MODE, int T>
__device__ inline void grid_small(const ProbDesc& P, const int4 it, int src_slot) {
  static_assert(T <= 8 && kSmallChunk <= 64, "eight taps and an entry per lane");
  constexpr int RG = kGridTile + T - 1;
  constexpr int DEG = KbDeg<R>::value;
  constexpr int NCELL = (RG * RG + 63) / 64;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  if (wave >= it.w) return;
  const int c = P.small_ids[it.z + wave];
  const int4 ch = P.chunks[c];
  const int2 ent = P.chunk_ent[c];
  const int box = P.slot_box[ch.w];
  const int ne = ent.y - ent.x;
  const int m = ent.x + (lane < ne ? lane : 0);             // the chunk's rows are contiguous
  R cr[DEG + 1];
  {
    const int tap = lane & 7;
    const R* __restrict__ poly = (const R*)P.kbpoly + (tap < T ? tap : 0) * (DEG + 1);
#pragma unroll
    for (int k = 0; k <= DEG; ++k) cr[k] = poly[k];
  }
  const V2<R> fm = ((const V2<R>*)P.vis_frac)[m];
  const int pkm = P.vis_k0[m];
  V4<R> u0, u1;
  (void)grid_channels<R, MODE>(P, m, ((const Cell<R>*)P.vis[src_slot])[m], u0, u1);

  const int ntg = P.ntile_side_g;
  const int t1 = ch.x / ntg, t2 = ch.x - t1 * ntg;
  const int b1 = t1 * kGridTile, b2 = t2 * kGridTile;
  const int lo1 = box & 255, lo2 = (box >> 16) & 255;
  const int bw = ((box >> 8) & 255) - lo1 + 1, area = bw * (((box >> 24) & 255) - lo2 + 1);
  int cell[NCELL];                                  // region offsets o1 | o2 << 8 of the lane's cells
#pragma unroll
  for (int k = 0; k < NCELL; ++k) {
    const int q = lane + 64 * k, a = q / bw;
    cell[k] = (lo1 + q - a * bw) | ((lo2 + a) << 8);
  }
  R acc[NCELL][8];
#pragma unroll
  for (int k = 0; k < NCELL; ++k)
#pragma unroll
    for (int h = 0; h < 8; ++h) acc[k][h] = R(0);
  for (int e = 0; e < ne; ++e) {
    const V2<R> f = lane_value(fm, e);
    const int pk = lane_value(pkm, e);
    const V4<R> v0 = lane_value(u0, e), v1 = lane_value(u1, e);
    const R u[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
    const R w = kb_tap<R, T>(R(2) * (lane < 8 ? f.x : f.y) - R(T - 1), cr);
    const int s1 = (pk >> 16) - b1, s2 = (pk & 0xffff) - b2;
#pragma unroll
    for (int k = 0; k < NCELL; ++k) {
      const int i = (cell[k] & 255) - s1, j = (cell[k] >> 8) - s2;
      const R wi = __shfl(w, i & 7), wj = __shfl(w, 8 + (j & 7));
      const R ww = ((unsigned)i < (unsigned)T && (unsigned)j < (unsigned)T) ? wi * wj : R(0);
#pragma unroll
      for (int h = 0; h < 8; ++h) acc[k][h] += ww * u[h];
    }
  }
  Cell<R>* __restrict__ dst = (Cell<R>*)P.gpart + (size_t)ch.w * RG * RG;
#pragma unroll
  for (int k = 0; k < NCELL; ++k) {
    if (lane + 64 * k >= area) break;
    Cell<R> o;
#pragma unroll
    for (int h = 0; h < 4; ++h) o.s[h] = cmk(acc[k][2 * h], acc[k][2 * h + 1]);
    dst[(cell[k] >> 8) * RG + (cell[k] & 255)] = o;
  }
}

// (FP64: the LDS holds one workgroup per CU, so two waves per SIMD and 256 registers, which
// keeps the FP64 accumulators out of scratch memory)
// (ce: the largest chunk of the launch's problems; the staging arrays after the accumulator hold
// ce entries)
template <typename R, int MODE, int T>
__global__ void __launch_bounds__(kGridThreads, sizeof(R) == 8 ? 2 : 4)
grid_kernel(const ProbDesc* __restrict__ descs, const int4* __restrict__ items, int src_slot, int use_cfac, int ce) {
  constexpr int RG = kGridTile + T - 1;            // tile plus halo
  __shared__ unsigned long long acc[8 * RG * RG];   // channel-major: acc[c][k2 offset][k1 offset]
  extern __shared__ __align__(16) unsigned char stage_raw[];
  V2<R>* sf = (V2<R>*)stage_raw;                  // staged fractional offsets
  V4<R>* su = (V4<R>*)(stage_raw + (size_t)ce * sizeof(V2<R>));   // staged mixed values, two V4 per entry
  __shared__ double red[2 * (kGridThreads / 64)];
  const int4 it = items[blockIdx.x];
  const ProbDesc& P = descs[it.x];
  if (it.y == kGridSmallItem) {    // up to eight small chunks, one per wave
    if (halted(P)) return;         // stopped by an adaptive run
    grid_small<R, MODE, T>(P, it, src_slot);
    return;
  }
  if (it.y == kGridFactorItem) {   // the factor item: the factor the column inverse FFT applies
    if (halted(P)) return;
    if (MODE == GR_DUAL) {
      const double v2 = block_sum_partials(P.partials, P.n_p6, red);
      if (threadIdx.x == 0) {
        const double vn = sqrt(v2);
        const double c = (vn > P.eps) ? P.rho2 * (1.0 - P.eps / vn) : 0.0;
        P.scal[SC_CFAC] = c;
        P.scal[SC_VNORM2] = v2;
        P.scal[SC_GFAC] = c;
      }
    } else if (threadIdx.x == 0) {
      P.scal[SC_GFAC] = use_cfac ? P.scal[SC_CFAC] : 1.0;
    }
    return;
  }
  // a chunk item carries its entry range; everything the chunk reads is requested before the
  // halt test so the loads are in flight together (a thread's entries are q and q + blockDim.x)
  static_assert(kChunkEntries <= 2 * kGridThreads, "two entries per thread");
  const int2 ent = make_int2(it.z, it.w);
  const int ne = ent.y - ent.x;
  int me[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int q = threadIdx.x + e * blockDim.x;
    me[e] = ent.x + (q < ne ? q : 0);                      // the chunk's rows are contiguous
  }
  const int4 ch = P.chunks[it.y];
  constexpr bool kPoly = sizeof(R) == 4;
  ChunkPre<R> pre;
  chunk_preload<R, T, kPoly>(P, ch, pre);
  if (halted(P)) return;                 // stopped by an adaptive run

  // stage the chunk's entries: offsets and gridded channels; sum the largest channel magnitude
  // of each for the fixed point
  const Cell<R>* __restrict__ bsrc = (const Cell<R>*)P.vis[src_slot];
  const V2<R>* __restrict__ frac = (const V2<R>*)P.vis_frac;
  V2<R> fe[2];
  Cell<R> be[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    fe[e] = frac[me[e]];
    be[e] = bsrc[me[e]];
  }
  for (int q = threadIdx.x; q < 8 * RG * RG; q += blockDim.x) acc[q] = 0ull;
  KSum bound;
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int q = threadIdx.x + e * blockDim.x;
    if (q >= ne) break;
    sf[q] = fe[e];
    V4<R> u0, u1;
    const R mx = grid_channels<R, MODE>(P, me[e], be[e], u0, u1);
    su[2 * q] = u0;
    su[2 * q + 1] = u1;
    bound.add((double)mx);
  }
  const double total = block_reduce(bound, red).value();      // includes a barrier
  grid_chunk<R, T, kPoly>(P, ch, sf, su, acc, fixed_exponent<R>(total), pre);
}

// ---------------------------------------------------------------------------------------------
// P6 + P7 in one pass (MODE GR_DUAL: Algorithm 1's dual B step and its gridding, DG_DUAL then
// GR_DUAL; GR_STOKES: Algorithm 3's data-term residual, DG_STOKES then GR_STOKES).  items: the gridding work list; its factor item does nothing here, since the
// column inverse FFT that follows derives the factor from this pass's partials.
//
// A chunk's rows all have their window start in its tile, so every tap they read lies in the
// tile plus its (T-1)-wide halo -- the region the chunk accumulates.  The region of the grid is
// staged in LDS (in the memory the accumulation takes afterwards); each row is de-gridded there
// by one thread, stored (Bv, or the residual) and staged for the gridding of the same chunk,
// and the FP64 squared norms of the chunk go to its pair of chunk_partials.
// (FP64: the LDS holds one workgroup per CU, so two waves per SIMD and 256 registers)
template <typename R, int MODE, int T>
__global__ void __launch_bounds__(kGridThreads, sizeof(R) == 8 ? 2 : 4)
degrid_grid_kernel(const ProbDesc* __restrict__ descs, const int4* __restrict__ items, int src_slot, int out_slot,
                   int ce) {
  constexpr int RG = kGridTile + T - 1;
  constexpr int DG = MODE == GR_STOKES ? DG_STOKES : DG_DUAL;
  __shared__ unsigned long long acc[8 * RG * RG];   // first the grid window (RG x RG cells)
  extern __shared__ __align__(16) unsigned char stage_raw[];
  V2<R>* sf = (V2<R>*)stage_raw;
  V4<R>* su = (V4<R>*)(stage_raw + (size_t)ce * sizeof(V2<R>));
  __shared__ double red[2 * (kGridThreads / 64)];
  static_assert(sizeof(Cell<R>) <= 8 * sizeof(unsigned long long), "window fits the accumulator");
  const int4 it = items[blockIdx.x];
  const ProbDesc& P = descs[it.x];
  if (halted(P) || it.y < 0) return;
  const int4 ch = P.chunks[it.y];
  const int2 ent = make_int2(it.z, it.w);       // the chunk's entry range, carried by the item
  ChunkPre<R> pre;
  chunk_preload<R, T, false>(P, ch, pre);
  const int K = P.K, ntg = P.ntile_side_g;
  const int t1 = ch.x / ntg, t2 = ch.x - t1 * ntg;
  const int b1 = t1 * kGridTile, b2 = t2 * kGridTile;
  // a thread's entries are q and q + blockDim.x: their indices, window starts and offsets are
  // loaded first, so that those loads and the window's are in flight together
  static_assert(kChunkEntries <= 2 * kGridThreads, "two entries per thread");
  const int ne = ent.y - ent.x;
  const V2<R>* __restrict__ frac = (const V2<R>*)P.vis_frac;
  int me[2], pke[2];
  V2<R> fe[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int q = threadIdx.x + e * blockDim.x;
    me[e] = ent.x + (q < ne ? q : 0);                      // the chunk's rows are contiguous
  }
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    pke[e] = P.vis_k0[me[e]];
    fe[e] = frac[me[e]];
  }
  Cell<R>* win = (Cell<R>*)acc;
  const Cell<R>* __restrict__ grid = (const Cell<R>*)P.grid;
  stage_lds<(RG * RG + kGridThreads - 1) / kGridThreads>(win, RG * RG, [&](int q) {
    const int a = q / RG, b = q - a * RG;                     // a: k2 offset, b: k1 offset
    return grid[(size_t)((b2 + a) & (K - 1)) * K + ((b1 + b) & (K - 1))];
  });
  __syncthreads();

  Cell<R>* __restrict__ out = (Cell<R>*)P.vis[out_slot];
  KSum bound, norm;
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int q = threadIdx.x + e * blockDim.x;
    if (q >= ne) break;
    const int m = me[e], pk = pke[e];
    const V2<R> f = fe[e];
    R w1[T], w2[T];
    kb_weights<R, T>(f.x, (const R*)P.kbpoly, w1);
    kb_weights<R, T>(f.y, (const R*)P.kbpoly, w2);
    cplx<R> v[4];
    interpolate<R, T>(win, RG, (pk >> 16) - b1, (pk & 0xffff) - b2, w1, w2, v);
    const Cell<R> o = degrid_row<R, DG>(P, m, v, src_slot, norm);
    out[m] = o;
    sf[q] = f;
    V4<R> u0, u1;
    const R mx = grid_channels<R, MODE>(P, m, o, u0, u1);
    su[2 * q] = u0;
    su[2 * q + 1] = u1;
    bound.add((double)mx);
  }
  const KSum nt = block_reduce(norm, red);                     // barriers: the window is done
  if (threadIdx.x == 0) {
    double* pp = chunk_partials(P);
    pp[2 * ch.w] = nt.s;
    pp[2 * ch.w + 1] = nt.c;
  }
  const double total = block_reduce(bound, red).value();
  for (int q = threadIdx.x; q < 8 * RG * RG; q += blockDim.x) acc[q] = 0ull;
  __syncthreads();
  grid_chunk<R, T, false>(P, ch, sf, su, acc, fixed_exponent<R>(total), pre);
}

// dynamic LDS of the gridding kernels: the staged offsets and mixed values of ce entries
template <typename R> size_t grid_stage_bytes(int ce) { return (size_t)ce * (sizeof(V2<R>) + 2 * sizeof(V4<R>)); }

template <typename R, int T>
void launch_grid_t(int mode, const LaunchArgs& a, int src_slot, int use_cfac) {
  const dim3 grid(a.nitems), block(kGridThreads);
  const int ce = a.grid_ce;
  const size_t shm = grid_stage_bytes<R>(ce);
  if (mode == GR_DUAL) {
    hipLaunchKernelGGL((grid_kernel<R, GR_DUAL, T>), grid, block, shm, a.stream, a.descs, a.items, src_slot, use_cfac, ce);
  } else if (mode == GR_STOKES) {
    hipLaunchKernelGGL((grid_kernel<R, GR_STOKES, T>), grid, block, shm, a.stream, a.descs, a.items, src_slot, use_cfac, ce);
  } else {
    hipLaunchKernelGGL((grid_kernel<R, GR_PLAIN, T>), grid, block, shm, a.stream, a.descs, a.items, src_slot, use_cfac, ce);
  }
}

// taps: the kernel support T of every problem in the launch (4, 6 or 8)
template <typename R>
void launch_grid(int mode, const LaunchArgs& a, int taps, int src_slot, int use_cfac) {
  if (a.nitems <= 0) return;
  if (taps == 4) launch_grid_t<R, 4>(mode, a, src_slot, use_cfac);
  else if (taps == 6) launch_grid_t<R, 6>(mode, a, src_slot, use_cfac);
  else launch_grid_t<R, 8>(mode, a, src_slot, use_cfac);
}

template <typename R, int T>
void launch_degrid_grid_t(int mode, const LaunchArgs& a, int src_slot, int out_slot) {
  const dim3 grid(a.nitems), block(kGridThreads);
  const int ce = a.grid_ce;
  const size_t shm = grid_stage_bytes<R>(ce);
  if (mode == GR_STOKES) {
    hipLaunchKernelGGL((degrid_grid_kernel<R, GR_STOKES, T>), grid, block, shm, a.stream, a.descs, a.items, src_slot,
                       out_slot, ce);
  } else {
    hipLaunchKernelGGL((degrid_grid_kernel<R, GR_DUAL, T>), grid, block, shm, a.stream, a.descs, a.items, src_slot,
                       out_slot, ce);
  }
}

template <typename R>
void launch_degrid_grid(int mode, const LaunchArgs& a, int taps, int src_slot, int out_slot) {
  if (a.nitems <= 0) return;
  if (taps == 4) launch_degrid_grid_t<R, 4>(mode, a, src_slot, out_slot);
  else if (taps == 6) launch_degrid_grid_t<R, 6>(mode, a, src_slot, out_slot);
  else launch_degrid_grid_t<R, 8>(mode, a, src_slot, out_slot);
}

// Raise the dynamic-LDS limit of the de-grid / grid kernels once, outside any graph capture.
template <typename R, int T>
void set_degrid_limits_t(int max_ts) {
  const int shm_st = (int)grid_stage_bytes<R>(kChunkEntries);
  hip_check(hipFuncSetAttribute((const void*)grid_kernel<R, GR_DUAL, T>, hipFuncAttributeMaxDynamicSharedMemorySize, shm_st), "attr");
  hip_check(hipFuncSetAttribute((const void*)grid_kernel<R, GR_PLAIN, T>, hipFuncAttributeMaxDynamicSharedMemorySize, shm_st), "attr");
  hip_check(hipFuncSetAttribute((const void*)grid_kernel<R, GR_STOKES, T>, hipFuncAttributeMaxDynamicSharedMemorySize, shm_st), "attr");
  hip_check(hipFuncSetAttribute((const void*)degrid_grid_kernel<R, GR_DUAL, T>, hipFuncAttributeMaxDynamicSharedMemorySize, shm_st), "attr");
  hip_check(hipFuncSetAttribute((const void*)degrid_grid_kernel<R, GR_STOKES, T>, hipFuncAttributeMaxDynamicSharedMemorySize, shm_st), "attr");
  const int W = max_ts + T - 1;
  const int shm_dg = W * W * (int)sizeof(Cell<R>);
  hip_check(hipFuncSetAttribute((const void*)degrid_kernel<R, DG_DUAL, T>, hipFuncAttributeMaxDynamicSharedMemorySize, shm_dg), "attr");
  hip_check(hipFuncSetAttribute((const void*)degrid_kernel<R, DG_FORWARD, T>, hipFuncAttributeMaxDynamicSharedMemorySize, shm_dg), "attr");
  hip_check(hipFuncSetAttribute((const void*)degrid_kernel<R, DG_RESIDUAL, T>, hipFuncAttributeMaxDynamicSharedMemorySize, shm_dg), "attr");
  hip_check(hipFuncSetAttribute((const void*)degrid_kernel<R, DG_STOKES, T>, hipFuncAttributeMaxDynamicSharedMemorySize, shm_dg), "attr");
}

// Set once per device for every tap count, at the largest de-grid tile (hipFuncSetAttribute is
// a device-wide setting, so later engines and batches need not repeat it).
template <typename R>
void set_grid_kernel_limits(int /*max_ts*/, int /*taps*/) {
  static std::mutex mu;
  static std::set<int> done;
  int dev = 0;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  std::lock_guard<std::mutex> lk(mu);
  if (done.count(dev)) return;
  set_degrid_limits_t<R, 4>(kMaxDegridTile);
  set_degrid_limits_t<R, 6>(kMaxDegridTile);
  set_degrid_limits_t<R, 8>(kMaxDegridTile);
  done.insert(dev);
}

template void set_grid_kernel_limits<float>(int, int);
template void set_grid_kernel_limits<double>(int, int);
template void launch_degrid<float>(int, const LaunchArgs&, int, int, int, int);
template void launch_degrid<double>(int, const LaunchArgs&, int, int, int, int);
template void launch_grid<float>(int, const LaunchArgs&, int, int, int);
template void launch_grid<double>(int, const LaunchArgs&, int, int, int);
template void launch_degrid_grid<float>(int, const LaunchArgs&, int, int, int);
template void launch_degrid_grid<double>(int, const LaunchArgs&, int, int, int);


}  // namespace psara
