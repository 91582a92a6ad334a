// SARA dictionary Psi = (1/sqrt(nb)) [Dirac, Db1..Db8] (Sec. 3.1) and the sparsity dual
// update of Algorithm 1 (A~ = A + rho1 Psi^dagger X; A = A~ - rho1 T_{gW/rho1}(A~/rho1),
// which is clip(A~, -gW, gW) for the soft-thresholding of eq. soft_thresh).
//
// Each wavelet basis is an orthonormal periodised 2-D DWT stored in the in-place Mallat
// layout.  One launch processes one level of every wavelet basis: a workgroup owns an
// output tile of the four sub-bands, stages the input region it needs (tile plus a filter
// halo, wrapped periodically, which also covers filters longer than the signal at coarse
// levels) in LDS, filters the rows into LDS and then the columns, and applies the
// requested per-coefficient operation at once, so coefficients never round-trip through
// memory:
//   AM_DUAL      A = clip(A + rho1 c, -gW, gW)
//   AM_STORE     out = c
//   AM_REWEIGHT  gW = gamma delta / (delta + |c|)    (eq. weights)
//   AM_OBJECTIVE partial sums of gW |c|               (weighted l1 norm, / gamma on the host)
//   AM_MOMENTS   partial sums of c and c^2
//   AM_MAXABS    partial maxima of |c|                 (the data-driven gamma)
// with c the normalised coefficient.  Intermediate low-low bands go to a per-basis
// scratch array.  Synthesis mirrors this from the coarsest level down; its last level sums
// every wavelet basis of a tile in registers and writes the image once.  The Dirac part of
// the dual update is pointwise and is fused into the primal kernel instead.
//
// The filter length F (2p for Db_p) is a template parameter of the filtering code, so the
// tap loops unroll and the taps live in registers; each kernel switches on the basis's F.
#include "common.hpp"
#include "launch.hpp"

namespace psara {

template <typename R>
__device__ inline void v4_fma(V4<R>& acc, R w, const V4<R>& x) {
  acc.x += w * x.x; acc.y += w * x.y; acc.z += w * x.z; acc.w += w * x.w;
}
template <typename R>
__device__ inline V4<R> v4_zero() { V4<R> v; v.x = v.y = v.z = v.w = R(0); return v; }
// component-wise load (keeps the destination in registers where a struct copy may not)
template <typename R>
__device__ __forceinline__ void ld4(V4<R>& d, const V4<R>* __restrict__ p) {
  d.x = p->x; d.y = p->y; d.z = p->z; d.w = p->w;
}

// Low-pass taps h and the quadrature-mirror high-pass g[j] = (-1)^j h[F-1-j] of one basis.
template <typename R, int F>
struct Taps {
  R h[F], g[F];
  __device__ explicit Taps(const R* __restrict__ f) {
#pragma unroll
    for (int j = 0; j < F; ++j) h[j] = f[j];
#pragma unroll
    for (int j = 0; j < F; ++j) g[j] = (j & 1) ? -h[F - 1 - j] : h[F - 1 - j];
  }
};

// Expands CALL(F) for the run-time filter length of a basis (Db1..Db8).
#define PSARA_FILTER_SWITCH(Fval, CALL) \
  switch (Fval) {                       \
    case 2: CALL(2); break;             \
    case 4: CALL(4); break;             \
    case 6: CALL(6); break;             \
    case 8: CALL(8); break;             \
    case 10: CALL(10); break;           \
    case 12: CALL(12); break;           \
    case 14: CALL(14); break;           \
    default: CALL(16); break;           \
  }

template <typename R, int MODE>
__device__ inline void apply_coef(const ProbDesc& P, int out_coef, size_t idx, V4<R> raw, KSum& k1, KSum& k2) {
  const R nm = R(P.norm);
  V4<R> c;
  c.x = raw.x * nm; c.y = raw.y * nm; c.z = raw.z * nm; c.w = raw.w * nm;
  if (MODE == AM_DUAL) {
    V4<R>* A = (V4<R>*)P.coef[COEF_A];
    const V4<R> gw = ((const V4<R>*)P.coef[COEF_GW])[idx];
    V4<R> a = A[idx];
    const R r1 = R(P.rho1);
    a.x = fmin(fmax(a.x + r1 * c.x, -gw.x), gw.x);
    a.y = fmin(fmax(a.y + r1 * c.y, -gw.y), gw.y);
    a.z = fmin(fmax(a.z + r1 * c.z, -gw.z), gw.z);
    a.w = fmin(fmax(a.w + r1 * c.w, -gw.w), gw.w);
    A[idx] = a;
  } else if (MODE == AM_STORE) {
    ((V4<R>*)P.coef[out_coef])[idx] = c;
  } else if (MODE == AM_REWEIGHT) {
    const R d = R(P.delta), g = R(P.gamma);
    V4<R> w;
    w.x = g * d / (d + fabs(c.x)); w.y = g * d / (d + fabs(c.y));
    w.z = g * d / (d + fabs(c.z)); w.w = g * d / (d + fabs(c.w));
    ((V4<R>*)P.coef[COEF_GW])[idx] = w;
  } else if (MODE == AM_OBJECTIVE) {
    const V4<R> gw = ((const V4<R>*)P.coef[COEF_GW])[idx];
    k1.add((double)gw.x * fabs((double)c.x));
    k1.add((double)gw.y * fabs((double)c.y));
    k1.add((double)gw.z * fabs((double)c.z));
    k1.add((double)gw.w * fabs((double)c.w));
  } else if (MODE == AM_MAXABS) {
    k1.s = fmax(k1.s, (double)fmax(fmax(fabs(c.x), fabs(c.y)), fmax(fabs(c.z), fabs(c.w))));
  } else {
    k1.add((double)c.x); k1.add((double)c.y); k1.add((double)c.z); k1.add((double)c.w);
    k2.add((double)c.x * c.x); k2.add((double)c.y * c.y); k2.add((double)c.z * c.z); k2.add((double)c.w * c.w);
  }
}

__device__ inline double block_max(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < (int)((blockDim.x + 63) >> 6); ++w) r = fmax(r, red[w]);
  return r;
}

// the dual update clip(A + rho1 c, -gW, gW) on prefetched A and gW
template <typename R>
__device__ inline V4<R> dual_clip(V4<R> a, const V4<R>& gw, const V4<R>& raw, R r1n) {
  a.x = fmin(fmax(a.x + r1n * raw.x, -gw.x), gw.x);
  a.y = fmin(fmax(a.y + r1n * raw.y, -gw.y), gw.y);
  a.z = fmin(fmax(a.z + r1n * raw.z, -gw.z), gw.z);
  a.w = fmin(fmax(a.w + r1n * raw.w, -gw.w), gw.w);
  return a;
}

template <typename R>
__device__ inline void write_partials(const ProbDesc& P, int part, const KSum& k1, const KSum& k2, int two, double* red) {
  double* gen = P.partials + 2 * (size_t)P.n_p6;
  if (two < 0) {                                   // maximum
    const double m = block_max(k1.s, red);
    if (threadIdx.x == 0) { gen[2 * part] = m; gen[2 * part + 1] = 0.0; }
    return;
  }
  const KSum t1 = block_reduce(k1, red);
  if (threadIdx.x == 0) { gen[2 * part] = t1.s; gen[2 * part + 1] = t1.c; }
  if (two) {
    const KSum t2 = block_reduce(k2, red);
    if (threadIdx.x == 0) { gen[2 * (part + P.gen_stride)] = t2.s; gen[2 * (part + P.gen_stride) + 1] = t2.c; }
  }
}

// ---------------------------------------------------------------------------------------------
// Analysis of level `level` (1 = finest) for every wavelet basis.
// items: {prob, wavelet index, tile, partial index}; tile side dwt_ana_tile(h) per band.
// TOM is the largest tile side among the launch's items: the LDS buffers are sized for it, so a
// launch whose problems all use 8-wide tiles holds 22 KB (FP32) instead of 57 KB per workgroup.
// The row pass's results overwrite the staged input (rowt aliases in: the pass holds its
// outputs in registers across a barrier), so a workgroup needs one buffer; with SEP the row
// results have a buffer of their own, and the staged input outlives the pass (the level-1 items
// that run every basis over one staged region).
template <typename R, int TOM, bool SEP = false> struct AnaSmem {
  static constexpr int TO = TOM;
  static constexpr int IN = 2 * TO + kMaxFilter - 2;
  V4<R> in[IN * IN];
  V4<R> rt[SEP ? IN * 2 * TO : 1];
  __device__ V4<R>* rowt() { return SEP ? rt : in; }
};

// Where an analysis output tile lies: the level's band side m (input) and h (output), the tile
// side to (a power of two) and the tile's first output row o1 and column o2.
struct AnaTile {
  int m, h, to, lto, o1, o2;
};
template <typename R>
__device__ inline AnaTile ana_tile(const ProbDesc& P, int level, int tile) {
  AnaTile t;
  t.m = P.n >> (level - 1);
  t.h = t.m >> 1;
  t.to = dwt_ana_tile<R>(t.h, (P.ana_wide & kAnaWide) != 0);
  t.lto = lg2(t.to);
  const int tps = t.h >> t.lto;
  t.o1 = (tile >> lg2(tps)) * t.to;
  t.o2 = (tile & (tps - 1)) * t.to;
  return t;
}

// Stages the in x in input elements of a tile (from row 2 o1, column 2 o2 of the m x m band src,
// wrapped periodically) into sm.in as rows of in elements.
template <typename R, class Smem>
__device__ inline void ana_stage(Smem& sm, const V4<R>* __restrict__ src, const AnaTile& g, int in) {
  const float rin = 1.0f / (float)in;
  for (int q = threadIdx.x; q < in * in; q += blockDim.x) {
    const int a = small_div(q, rin), b = q - a * in;
    sm.in[q] = src[(size_t)((2 * g.o1 + a) & (g.m - 1)) * g.m + ((2 * g.o2 + b) & (g.m - 1))];
  }
}

// One basis w over one output tile.  ins = 0: stages the tile's input for this filter first;
// otherwise the input is staged already, as rows of ins elements (ins >= 2 to + F - 2).
template <typename R, int MODE, int F, int TOM, bool SEP>
__device__ __forceinline__ void analysis_body(const ProbDesc& P, AnaSmem<R, TOM, SEP>& sm, int w, int level, int tile,
                                              int src_slot, int out_coef, KSum& k1, KSum& k2, int ins) {
  const Taps<R, F> t((const R*)P.filters + w * kMaxFilter);
  const int n = P.n;
  const AnaTile g = ana_tile<R>(P, level, tile);
  const int h = g.h, to = g.to, lto = g.lto, o1 = g.o1, o2 = g.o2;
  const int in = 2 * to + F - 2;                   // input rows and columns this filter reads
  const size_t base = (size_t)(P.has_dirac + w) * n * n;
  const bool last = (level == P.levels);
  constexpr int NPF = (TOM * 2 * TOM + 255) / 256;
  if (ins == 0) {
    const V4<R>* __restrict__ src = (level == 1)
        ? (const V4<R>*)P.img[src_slot]
        : (const V4<R>*)P.ll + (size_t)w * P.ll_stride + P.ll_off[level - 1];
    ana_stage<R>(sm, src, g, in);
    ins = in;
    __syncthreads();
  }
  // rows: along the column index, into registers, then over the staged input
  constexpr int NQ = (AnaSmem<R, TOM, SEP>::IN * TOM + 255) / 256;
  V4<R> ra[NQ], rd[NQ];
#pragma unroll
  for (int u = 0; u < NQ; ++u) {
    const int q = threadIdx.x + u * 256;
    if (q < in * to) {
      const int a = q >> lto, k = q & (to - 1);
      V4<R> sa = v4_zero<R>(), sd = v4_zero<R>();
      const V4<R>* row = sm.in + a * ins + 2 * k;
#pragma unroll
      for (int j = 0; j < F; ++j) { const V4<R> x = row[j]; v4_fma(sa, t.h[j], x); v4_fma(sd, t.g[j], x); }
      ra[u] = sa;
      rd[u] = sd;
    }
  }
  // the duals and thresholds this thread updates, requested now so their latency overlaps the
  // column filtering
  V4<R> pa[NPF][2], pg[NPF][2];
  if (MODE == AM_DUAL) {
    const V4<R>* __restrict__ A = (const V4<R>*)P.coef[COEF_A];
    const V4<R>* __restrict__ GW = (const V4<R>*)P.coef[COEF_GW];
#pragma unroll
    for (int u = 0; u < NPF; ++u) {
      const int q = threadIdx.x + u * 256;
      if (q < to * 2 * to) {
        const int kr = q >> (lto + 1), c = q & (2 * to - 1);
        const int col = (c < to) ? o2 + c : h + o2 + (c - to);
        const size_t ia = base + (size_t)(o1 + kr) * n + col, id = base + (size_t)(h + o1 + kr) * n + col;
        if (!(c < to && !last)) { pa[u][0] = A[ia]; pg[u][0] = GW[ia]; }
        pa[u][1] = A[id]; pg[u][1] = GW[id];
      }
    }
  }
  __syncthreads();                       // every thread is done reading the staged input
  V4<R>* rowt = sm.rowt();
#pragma unroll
  for (int u = 0; u < NQ; ++u) {
    const int q = threadIdx.x + u * 256;
    if (q < in * to) {
      const int a = q >> lto, k = q & (to - 1);
      rowt[a * (2 * to) + k] = ra[u];
      rowt[a * (2 * to) + to + k] = rd[u];
    }
  }
  __syncthreads();
  // columns, then the per-coefficient operation
  V4<R>* llout = (V4<R>*)P.ll + (size_t)w * P.ll_stride + P.ll_off[level];
  V4<R>* __restrict__ Aw = (V4<R>*)P.coef[COEF_A];
  const R r1n = R(P.rho1) * R(P.norm);
#pragma unroll
  for (int u = 0; u < NPF; ++u) {
    const int q = threadIdx.x + u * 256;
    if (q < to * 2 * to) {
      const int kr = q >> (lto + 1), c = q & (2 * to - 1);
      V4<R> ca = v4_zero<R>(), cd = v4_zero<R>();
#pragma unroll
      for (int j = 0; j < F; ++j) {
        const V4<R> x = rowt[(2 * kr + j) * (2 * to) + c];
        v4_fma(ca, t.h[j], x);
        v4_fma(cd, t.g[j], x);
      }
      const int col = (c < to) ? o2 + c : h + o2 + (c - to);
      const int rowa = o1 + kr, rowd = h + o1 + kr;
      const size_t ia = base + (size_t)rowa * n + col, id = base + (size_t)rowd * n + col;
      if (MODE == AM_DUAL) {
        if (c < to && !last) llout[(size_t)rowa * h + col] = ca;     // low-low band feeds the next level
        else Aw[ia] = dual_clip(pa[u][0], pg[u][0], ca, r1n);
        Aw[id] = dual_clip(pa[u][1], pg[u][1], cd, r1n);
      } else {
        if (c < to && !last) llout[(size_t)rowa * h + col] = ca;
        else apply_coef<R, MODE>(P, out_coef, ia, ca, k1, k2);
        apply_coef<R, MODE>(P, out_coef, id, cd, k1, k2);
      }
    }
  }
}

// items: {prob, basis, tile, partial index}; with SEP also {prob, kAllBases, tile, -} at level 1:
// every basis over the tile, the image region staged once with the halo of the longest filter
// (the bases of a level-1 tile all read the same image region; deeper levels read each basis's
// own low-low band).
template <typename R, int MODE, int TOM, bool SEP>
__global__ void __launch_bounds__(256)
analysis_kernel(const ProbDesc* __restrict__ descs, const int4* __restrict__ items, int level, int src_slot, int out_coef) {
  __shared__ AnaSmem<R, TOM, SEP> sm;
  __shared__ double red[8];
  const int4 it = items[blockIdx.x];
  const ProbDesc& P = descs[it.x];
  if (halted(P)) return;                 // stopped by an adaptive run
  KSum k1, k2;
  if (SEP && it.y == kAllBases) {
    const AnaTile g = ana_tile<R>(P, 1, it.z);
    const int ins = 2 * g.to + kMaxFilter - 2;
    ana_stage<R>(sm, (const V4<R>*)P.img[src_slot], g, ins);
    __syncthreads();
    for (int w = 0; w < P.nwav; ++w) {
#define PSARA_ANA(FF) analysis_body<R, MODE, FF, TOM, SEP>(P, sm, w, 1, it.z, src_slot, out_coef, k1, k2, ins)
      PSARA_FILTER_SWITCH(P.wav_len[w], PSARA_ANA)
#undef PSARA_ANA
    }
    return;
  }
  const int w = it.y;
#define PSARA_ANA(FF) analysis_body<R, MODE, FF, TOM, SEP>(P, sm, w, level, it.z, src_slot, out_coef, k1, k2, 0)
  PSARA_FILTER_SWITCH(P.wav_len[w], PSARA_ANA)
#undef PSARA_ANA
  if (MODE == AM_OBJECTIVE || MODE == AM_MOMENTS || MODE == AM_MAXABS)
    write_partials<R>(P, it.w, k1, k2, MODE == AM_MAXABS ? -1 : MODE == AM_MOMENTS, red);
}

// Dirac block for the non-dual modes.  items: {prob, block of 256 pixels, -, partial index}
template <typename R, int MODE>
__global__ void __launch_bounds__(256)
dirac_kernel(const ProbDesc* __restrict__ descs, const int4* __restrict__ items, int src_slot, int out_coef) {
  __shared__ double red[8];
  const int4 it = items[blockIdx.x];
  const ProbDesc& P = descs[it.x];
  if (halted(P)) return;                 // stopped by an adaptive run
  const int N = P.n * P.n;
  const int p = it.y * 256 + threadIdx.x;
  KSum k1, k2;
  if (p < N) apply_coef<R, MODE>(P, out_coef, (size_t)p, ((const V4<R>*)P.img[src_slot])[p], k1, k2);
  if (MODE == AM_OBJECTIVE || MODE == AM_MOMENTS || MODE == AM_MAXABS)
    write_partials<R>(P, it.w, k1, k2, MODE == AM_MAXABS ? -1 : MODE == AM_MOMENTS, red);
}

// ---------------------------------------------------------------------------------------------
// Synthesis of one to x to output tile (to = dwt_syn_tile) of the level-(level-1) low-low band
// (the image at level 1) of one basis.  The four band windows are fetched for the longest
// filter (KWM = to/2 + kMaxFilter/2 - 1 coefficients per side, starting kMaxFilter/2 - 1 before
// the tile's first coefficient); a basis with F taps uses the sub-window at offset
// kMaxFilter/2 - F/2.  The fetch goes through registers (one element of each band window per
// thread) so the final level can issue the next basis's loads before filtering the current one.
template <typename R>
struct SynSmem {
  static constexpr int TS = dwt_syn_tile<R>(1 << 30);
  static constexpr int KWM = TS / 2 + kMaxFilter / 2 - 1;
  V4<R> band[4][KWM * KWM];      // LL, HL (top-right), LH (bottom-left), HH windows
  V4<R> cola[TS * KWM], cold[TS * KWM];
};

template <typename R>
__device__ __forceinline__ void syn_fetch(const ProbDesc& P, int w, int level, int o1, int o2, int to, int src_coef,
                                          V4<R>* pre) {
  constexpr int KWM = SynSmem<R>::KWM;
  static_assert(KWM * KWM <= 256, "one window element per thread and band");
  const int n = P.n, h = (n >> (level - 1)) >> 1;
  const int kw = to / 2 + kMaxFilter / 2 - 1;
  const int e = threadIdx.x, a = e / KWM, b = e - a * KWM;
  if (e < KWM * KWM && a < kw && b < kw) {
    const int r = (o1 / 2 - (kMaxFilter / 2 - 1) + a) & (h - 1), c = (o2 / 2 - (kMaxFilter / 2 - 1) + b) & (h - 1);
    const V4<R>* __restrict__ A = (const V4<R>*)P.coef[src_coef] + (size_t)(P.has_dirac + w) * n * n;
    const V4<R>* l0 = (level == P.levels) ? A + (size_t)r * n + c
        : (const V4<R>*)P.ll + (size_t)w * P.ll_stride + P.ll_off[level] + (size_t)r * h + c;
    ld4(pre[0], l0);
    ld4(pre[1], A + (size_t)r * n + h + c);
    ld4(pre[2], A + (size_t)(h + r) * n + c);
    ld4(pre[3], A + (size_t)(h + r) * n + h + c);
  }
}

template <typename R>
__device__ __forceinline__ void syn_store(SynSmem<R>& sm, const V4<R>* pre) {
  constexpr int KWM = SynSmem<R>::KWM;
  if (threadIdx.x < KWM * KWM) {
#pragma unroll
    for (int u = 0; u < 4; ++u) sm.band[u][threadIdx.x] = pre[u];
  }
}

// Filters the staged windows into acc.  Output rows (columns) come in pairs 2k, 2k+1 that read
// the same coefficients, the even one through the even taps and the odd one through the odd
// taps, so one thread computes both.  acc[2u], acc[2u+1]: the pair q = threadIdx.x + 256 u of
// the to x to tile, row q / (to/2), columns 2 (q % (to/2)) and 2 (q % (to/2)) + 1.
template <int F, typename R>
__device__ __forceinline__ void syn_filter(const ProbDesc& P, SynSmem<R>& sm, int w, int o1, int o2, int to, V4<R>* acc) {
  constexpr int KWM = SynSmem<R>::KWM;
  constexpr int NPAIR = (SynSmem<R>::TS * SynSmem<R>::TS / 2 + 255) / 256;
  const Taps<R, F> t((const R*)P.filters + w * kMaxFilter);
  const int off = kMaxFilter / 2 - F / 2;          // sub-window of this filter length
  const int kw = to / 2 + F / 2 - 1, th = to / 2;
  const float rkw = 1.0f / (float)kw;
  const int lth = lg2(th);
  const int ks1 = o1 / 2 - (kMaxFilter / 2 - 1), ks2 = o2 / 2 - (kMaxFilter / 2 - 1);
  __syncthreads();
  // inverse column transform (along the row index): row pairs at full resolution
  for (int q = threadIdx.x; q < th * kw; q += blockDim.x) {
    const int rp = small_div(q, rkw), b = q - rp * kw + off;
    const int a0 = (o1 >> 1) + rp - ks1;             // coefficient row of output rows 2rp, 2rp+1
    V4<R> sa0 = v4_zero<R>(), sd0 = v4_zero<R>(), sa1 = v4_zero<R>(), sd1 = v4_zero<R>();
#pragma unroll
    for (int jj = 0; jj < F / 2; ++jj) {
      const int a = a0 - jj;
      const V4<R> ll = sm.band[0][a * KWM + b], lh = sm.band[2][a * KWM + b];
      const V4<R> hl = sm.band[1][a * KWM + b], hh = sm.band[3][a * KWM + b];
      v4_fma(sa0, t.h[2 * jj], ll); v4_fma(sa0, t.g[2 * jj], lh);
      v4_fma(sd0, t.h[2 * jj], hl); v4_fma(sd0, t.g[2 * jj], hh);
      v4_fma(sa1, t.h[2 * jj + 1], ll); v4_fma(sa1, t.g[2 * jj + 1], lh);
      v4_fma(sd1, t.h[2 * jj + 1], hl); v4_fma(sd1, t.g[2 * jj + 1], hh);
    }
    sm.cola[(2 * rp) * KWM + b] = sa0;
    sm.cold[(2 * rp) * KWM + b] = sd0;
    sm.cola[(2 * rp + 1) * KWM + b] = sa1;
    sm.cold[(2 * rp + 1) * KWM + b] = sd1;
  }
  __syncthreads();
  // inverse row transform (along the column index): column pairs
#pragma unroll
  for (int u = 0; u < NPAIR; ++u) {
    const int q = threadIdx.x + u * 256;
    if (q < to * th) {
      const int ir = q >> lth, cp = q & (th - 1);
      const int b0 = (o2 >> 1) + cp - ks2;
      V4<R> s0 = acc[2 * u], s1 = acc[2 * u + 1];
#pragma unroll
      for (int jj = 0; jj < F / 2; ++jj) {
        const V4<R> ca = sm.cola[ir * KWM + b0 - jj], cd = sm.cold[ir * KWM + b0 - jj];
        v4_fma(s0, t.h[2 * jj], ca); v4_fma(s0, t.g[2 * jj], cd);
        v4_fma(s1, t.h[2 * jj + 1], ca); v4_fma(s1, t.g[2 * jj + 1], cd);
      }
      acc[2 * u] = s0;
      acc[2 * u + 1] = s1;
    }
  }
}

// Levels L..2: items {prob, wavelet index, tile, -}; writes the low-low band of level-1.
template <typename R>
__global__ void __launch_bounds__(256)
synthesis_kernel(const ProbDesc* __restrict__ descs, const int4* __restrict__ items, int level, int src_coef) {
  __shared__ SynSmem<R> sm;
  constexpr int NPAIR = (SynSmem<R>::TS * SynSmem<R>::TS / 2 + 255) / 256;
  const int4 it = items[blockIdx.x];
  const ProbDesc& P = descs[it.x];
  if (halted(P)) return;                 // stopped by an adaptive run
  const int w = it.y;
  const int m = P.n >> (level - 1);
  const int to = dwt_syn_tile<R>(m), tps = m / to, th = to / 2;
  const int lth = lg2(th);                         // powers of two
  const int o1 = (it.z >> lg2(tps)) * to, o2 = (it.z & (tps - 1)) * to;
  V4<R> acc[2 * NPAIR], pre[4];
#pragma unroll
  for (int u = 0; u < 2 * NPAIR; ++u) acc[u] = v4_zero<R>();
  syn_fetch<R>(P, w, level, o1, o2, to, src_coef, pre);
  syn_store<R>(sm, pre);
#define PSARA_SYN(FF) syn_filter<FF, R>(P, sm, w, o1, o2, to, acc)
  PSARA_FILTER_SWITCH(P.wav_len[w], PSARA_SYN)
  V4<R>* out = (V4<R>*)P.ll + (size_t)w * P.ll_stride + P.ll_off[level - 1];
#pragma unroll
  for (int u = 0; u < NPAIR; ++u) {
    const int q = threadIdx.x + u * 256;
    if (q < to * th) {
      V4<R>* o = out + (size_t)(o1 + (q >> lth)) * m + o2 + 2 * (q & (th - 1));
      o[0] = acc[2 * u];
      o[1] = acc[2 * u + 1];
    }
  }
}

// Level 1 of the wavelet bases in the item's mask, summed, times 1/sqrt(nb); optionally plus the
// Dirac block.  The next basis's windows are loaded into registers while the current one is
// filtered.  items: {prob, tile, part, mask of bases}; part 0 writes dst_slot (with the Dirac
// block), part 1 dst_slot2, so that a tile's bases can be split over two workgroups.
// (FP32: at most 96 registers, so five workgroups fit a CU; the kernel needs no more)
template <typename R>
__global__ void __launch_bounds__(256, sizeof(R) == 4 ? 5 : 1)
synthesis_final_kernel(const ProbDesc* __restrict__ descs, const int4* __restrict__ items, int src_coef, int dst_slot,
                       int add_dirac, int dst_slot2) {
  __shared__ SynSmem<R> sm;
  constexpr int NPAIR = (SynSmem<R>::TS * SynSmem<R>::TS / 2 + 255) / 256;
  const int4 it = items[blockIdx.x];
  const ProbDesc& P = descs[it.x];
  if (halted(P)) return;                 // stopped by an adaptive run
  const int n = P.n;
  const int to = dwt_syn_tile<R>(n), tps = n / to, th = to / 2;
  const int lth = lg2(th);                         // powers of two
  const int o1 = (it.y >> lg2(tps)) * to, o2 = (it.y & (tps - 1)) * to;
  V4<R> acc[2 * NPAIR], pre[4];
#pragma unroll
  for (int u = 0; u < 2 * NPAIR; ++u) acc[u] = v4_zero<R>();
  unsigned mask = (unsigned)it.w & ((1u << P.nwav) - 1u);
  int w = mask ? __builtin_ctz(mask) : -1;
  if (w >= 0) syn_fetch<R>(P, w, 1, o1, o2, to, src_coef, pre);
  while (w >= 0) {
    mask &= mask - 1u;
    const int wn = mask ? __builtin_ctz(mask) : -1;
    __syncthreads();                       // the previous basis's windows are no longer read
    syn_store<R>(sm, pre);
    if (wn >= 0) syn_fetch<R>(P, wn, 1, o1, o2, to, src_coef, pre);
    PSARA_FILTER_SWITCH(P.wav_len[w], PSARA_SYN)
    w = wn;
  }
#undef PSARA_SYN
  const R nm = R(P.norm);
  const V4<R>* dirac = (const V4<R>*)P.coef[src_coef];
  const bool first = it.z == 0;
  V4<R>* out = (V4<R>*)P.img[first ? dst_slot : dst_slot2];
#pragma unroll
  for (int u = 0; u < 2 * NPAIR; ++u) {
    const int q = threadIdx.x + (u >> 1) * 256;
    if (q < to * th) {
      const size_t idx = (size_t)(o1 + (q >> lth)) * n + o2 + 2 * (q & (th - 1)) + (u & 1);
      V4<R> s = acc[u];
      if (first && add_dirac && P.has_dirac) {
        const V4<R> d = dirac[idx];
        s.x += d.x; s.y += d.y; s.z += d.z; s.w += d.w;
      }
      s.x *= nm; s.y *= nm; s.z *= nm; s.w *= nm;
      out[idx] = s;
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Coarse levels c..L of one wavelet basis and one Stokes channel in a single workgroup: the
// low-low band entering level c (at most CoarseMax<R> on a side) is held in LDS; analysis runs
// level by level with the dual update of every coefficient, which also stays in LDS as the
// Mallat pyramid of the coarse levels; synthesis then runs back from level L to level c on
// the updated duals and leaves the low-low band of level c-1 in the level scratch, where the
// next synthesis launch reads it.  Replaces 2 (L - c + 1) small launches by one.
// items: {prob, wavelet index (-1: none), Stokes channel, first coarse level c}
template <typename R> struct CoarseMax { static constexpr int value = sizeof(R) == 4 ? 64 : 32; };

template <typename R>
__device__ inline R& chan(V4<R>& v, int c) { return c == 0 ? v.x : c == 1 ? v.y : c == 2 ? v.z : v.w; }

template <int F, typename R>
__device__ __forceinline__ void coarse_body(const ProbDesc& P, int w, int ch, int c_level, R* bufA, R* bufB, R* pyr,
                                            R* gw) {
  const Taps<R, F> t((const R*)P.filters + w * kMaxFilter);
  const int n = P.n, L = P.levels, nt = blockDim.x;
  R* __restrict__ ll = (R*)((V4<R>*)P.ll + (size_t)w * P.ll_stride);
  R* __restrict__ A = (R*)((V4<R>*)P.coef[COEF_A] + (size_t)(P.has_dirac + w) * n * n);
  const R* __restrict__ GW = (const R*)((const V4<R>*)P.coef[COEF_GW] + (size_t)(P.has_dirac + w) * n * n);
  const R r1n = R(P.rho1) * R(P.norm);
  const int m0 = n >> (c_level - 1);               // side of the coarse pyramid
  int m = m0;
  // every coarse band lies in the top-left m0 x m0 block of the basis: its duals (into pyr,
  // where the updated ones are kept) and thresholds are staged with the low-low band, so the
  // dual updates below read LDS only
  // (each thread's loads are all issued before its LDS stores, so they are in flight together)
  {
    constexpr int NS = (CoarseMax<R>::value * CoarseMax<R>::value + 511) / 512;
    R va[NS], vp[NS], vg[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const int q = threadIdx.x + u * nt;
      if (q < m * m) {
        const size_t g = (size_t)(q >> lg2(m0)) * n + (q & (m0 - 1));
        va[u] = ll[4 * (P.ll_off[c_level - 1] + q) + ch];
        vp[u] = A[4 * g + ch];
        vg[u] = GW[4 * g + ch];
      }
    }
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const int q = threadIdx.x + u * nt;
      if (q < m * m) {
        bufA[q] = va[u];
        pyr[q] = vp[u];
        gw[q] = vg[u];
      }
    }
  }
  __syncthreads();
  // ---- analysis c..L (bufA holds the m x m low-low band) ----
  for (int l = c_level; l <= L; ++l) {
    const int h = m >> 1;
    for (int q = threadIdx.x; q < m * h; q += nt) {          // rows: bufB[r][k] = a, bufB[r][h+k] = d
      const int r = q >> lg2(h), k = q & (h - 1);
      R sa = R(0), sd = R(0);
#pragma unroll
      for (int j = 0; j < F; ++j) {
        const R x = bufA[r * m + ((2 * k + j) & (m - 1))];
        sa += t.h[j] * x;
        sd += t.g[j] * x;
      }
      bufB[r * m + k] = sa;
      bufB[r * m + h + k] = sd;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < h * m; q += nt) {          // columns; q = (k, col)
      const int k = q >> lg2(m), col = q & (m - 1);
      R ca = R(0), cd = R(0);
#pragma unroll
      for (int j = 0; j < F; ++j) {
        const R x = bufB[((2 * k + j) & (m - 1)) * m + col];
        ca += t.h[j] * x;
        cd += t.g[j] * x;
      }
      // (k, col): low rows; (h + k, col): high rows
      if (col < h && l < L) {
        bufA[k * h + col] = ca;                              // next level's input
      } else {
        const int p = k * m0 + col;
        const R a = fmin(fmax(pyr[p] + r1n * ca, -gw[p]), gw[p]);
        A[4 * ((size_t)k * n + col) + ch] = a;
        pyr[p] = a;
      }
      const int p = (h + k) * m0 + col;
      const R d = fmin(fmax(pyr[p] + r1n * cd, -gw[p]), gw[p]);
      A[4 * ((size_t)(h + k) * n + col) + ch] = d;
      pyr[p] = d;
    }
    __syncthreads();
    m = h;
  }
  // ---- synthesis L..c on the updated duals (bufA: the h x h low-low input) ----
  {
    const int h = n >> L;
    for (int q = threadIdx.x; q < h * h; q += nt) bufA[q] = pyr[(q >> lg2(h)) * m0 + (q & (h - 1))];
  }
  __syncthreads();
  for (int l = L; l >= c_level; --l) {
    const int mo = n >> (l - 1), h = mo >> 1;
    // inverse column transform: bufB[ir][b] (b < h) from LL/LH, bufB[mo*h + ir*h + b] from HL/HH;
    // output rows 2r', 2r'+1 read the same coefficients through the even / odd taps
    for (int q = threadIdx.x; q < h * h; q += nt) {
      const int rp = q >> lg2(h), b = q & (h - 1);
      R sa0 = R(0), sd0 = R(0), sa1 = R(0), sd1 = R(0);
#pragma unroll
      for (int jj = 0; jj < F / 2; ++jj) {
        const int r = (rp - jj) & (h - 1);
        const R ll = bufA[r * h + b], lh = pyr[(h + r) * m0 + b];
        const R hl = pyr[r * m0 + h + b], hh = pyr[(h + r) * m0 + h + b];
        sa0 += t.h[2 * jj] * ll + t.g[2 * jj] * lh;
        sd0 += t.h[2 * jj] * hl + t.g[2 * jj] * hh;
        sa1 += t.h[2 * jj + 1] * ll + t.g[2 * jj + 1] * lh;
        sd1 += t.h[2 * jj + 1] * hl + t.g[2 * jj + 1] * hh;
      }
      bufB[(2 * rp) * h + b] = sa0;
      bufB[mo * h + (2 * rp) * h + b] = sd0;
      bufB[(2 * rp + 1) * h + b] = sa1;
      bufB[mo * h + (2 * rp + 1) * h + b] = sd1;
    }
    __syncthreads();
    // inverse row transform into bufA (mo x mo), column pairs
    for (int q = threadIdx.x; q < mo * h; q += nt) {
      const int ir = q >> lg2(h), cp = q & (h - 1);
      R s0 = R(0), s1 = R(0);
#pragma unroll
      for (int jj = 0; jj < F / 2; ++jj) {
        const int b = (cp - jj) & (h - 1);
        const R ca = bufB[ir * h + b], cd = bufB[mo * h + ir * h + b];
        s0 += t.h[2 * jj] * ca + t.g[2 * jj] * cd;
        s1 += t.h[2 * jj + 1] * ca + t.g[2 * jj + 1] * cd;
      }
      bufA[ir * mo + 2 * cp] = s0;
      bufA[ir * mo + 2 * cp + 1] = s1;
    }
    __syncthreads();
  }
  for (int q = threadIdx.x; q < m0 * m0; q += nt) ll[4 * (P.ll_off[c_level - 1] + q) + ch] = bufA[q];
}

template <typename R>
__global__ void __launch_bounds__(512)
coarse_kernel(const ProbDesc* __restrict__ descs, const int4* __restrict__ items) {
  constexpr int MM = CoarseMax<R>::value;
  __shared__ R bufA[MM * MM], bufB[MM * MM], pyr[MM * MM], gw[MM * MM];
  const int4 it = items[blockIdx.x];
  const ProbDesc& P = descs[it.x];
  if (halted(P) || it.y < 0) return;    // stopped by an adaptive run, or an empty basis place
#define PSARA_COARSE(FF) coarse_body<FF, R>(P, it.y, it.z, it.w, bufA, bufB, pyr, gw)
  PSARA_FILTER_SWITCH(P.wav_len[it.y], PSARA_COARSE)
#undef PSARA_COARSE
}

template <typename R>
int coarse_level(int n, int levels) {
  // first level >= 2 whose input low-low band fits the LDS buffers
  for (int c = 2; c <= levels; ++c)
    if ((n >> (c - 1)) <= CoarseMax<R>::value) return c;
  return levels + 1;
}

template <typename R>
void launch_coarse(const LaunchArgs& a) {
  if (a.nitems <= 0) return;
  hipLaunchKernelGGL((coarse_kernel<R>), dim3(a.nitems), dim3(512), 0, a.stream, a.descs, a.items);
}

template <typename R, int TOM>
void launch_analysis_t(int mode, int level, const LaunchArgs& a, int src_slot, int out_coef) {
  const dim3 g(a.nitems), b(256);
#define PSARA_ANAL(M) \
  hipLaunchKernelGGL((analysis_kernel<R, M, TOM, false>), g, b, 0, a.stream, a.descs, a.items, level, src_slot, out_coef)
  // (only the iterations' dual lists hold all-bases items, so only AM_DUAL needs the SEP kernel)
  const bool all_bases = (a.ana_wide & kAnaAllBases) != 0;
  switch (mode) {
    case AM_DUAL:
      if (all_bases) {
        hipLaunchKernelGGL((analysis_kernel<R, AM_DUAL, TOM, true>), g, b, 0, a.stream, a.descs, a.items, level, src_slot,
                           out_coef);
      } else {
        PSARA_ANAL(AM_DUAL);
      }
      break;
    case AM_STORE: PSARA_ANAL(AM_STORE); break;
    case AM_REWEIGHT: PSARA_ANAL(AM_REWEIGHT); break;
    case AM_OBJECTIVE: PSARA_ANAL(AM_OBJECTIVE); break;
    case AM_MAXABS: PSARA_ANAL(AM_MAXABS); break;
    default: PSARA_ANAL(AM_MOMENTS); break;
  }
#undef PSARA_ANAL
}

template <typename R>
void launch_analysis(int mode, int level, const LaunchArgs& a, int src_slot, int out_coef) {
  if (a.nitems <= 0) return;
  // the largest tile side among the launch's problems (an unknown largest side takes the widest)
  constexpr int kWide = dwt_ana_tile<R>(1 << 30);
  const int tom = a.max_n > 0 ? dwt_ana_tile<R>(a.max_n >> level, (a.ana_wide & kAnaWide) != 0) : kWide;
  if constexpr (kWide > 8) {
    if (tom > 8) { launch_analysis_t<R, kWide>(mode, level, a, src_slot, out_coef); return; }
  }
  launch_analysis_t<R, 8>(mode, level, a, src_slot, out_coef);
}

template <typename R>
void launch_dirac(int mode, const LaunchArgs& a, int src_slot, int out_coef) {
  if (a.nitems <= 0) return;
  const dim3 g(a.nitems), b(256);
  switch (mode) {
    case AM_STORE: hipLaunchKernelGGL((dirac_kernel<R, AM_STORE>), g, b, 0, a.stream, a.descs, a.items, src_slot, out_coef); break;
    case AM_REWEIGHT: hipLaunchKernelGGL((dirac_kernel<R, AM_REWEIGHT>), g, b, 0, a.stream, a.descs, a.items, src_slot, out_coef); break;
    case AM_OBJECTIVE: hipLaunchKernelGGL((dirac_kernel<R, AM_OBJECTIVE>), g, b, 0, a.stream, a.descs, a.items, src_slot, out_coef); break;
    case AM_MOMENTS: hipLaunchKernelGGL((dirac_kernel<R, AM_MOMENTS>), g, b, 0, a.stream, a.descs, a.items, src_slot, out_coef); break;
    case AM_MAXABS: hipLaunchKernelGGL((dirac_kernel<R, AM_MAXABS>), g, b, 0, a.stream, a.descs, a.items, src_slot, out_coef); break;
    default: hipLaunchKernelGGL((dirac_kernel<R, AM_DUAL>), g, b, 0, a.stream, a.descs, a.items, src_slot, out_coef); break;
  }
}

template <typename R>
void launch_synthesis(int level, int /*coarsest*/, const LaunchArgs& a, int src_coef, int /*dst_slot*/) {
  if (a.nitems <= 0) return;
  hipLaunchKernelGGL((synthesis_kernel<R>), dim3(a.nitems), dim3(256), 0, a.stream, a.descs, a.items, level, src_coef);
}

template <typename R>
void launch_synthesis_final(const LaunchArgs& a, int src_coef, int dst_slot, int add_dirac, int dst_slot2) {
  if (a.nitems <= 0) return;
  hipLaunchKernelGGL((synthesis_final_kernel<R>), dim3(a.nitems), dim3(256), 0, a.stream, a.descs, a.items, src_coef,
                     dst_slot, add_dirac, dst_slot2);
}

template void launch_analysis<float>(int, int, const LaunchArgs&, int, int);
template void launch_analysis<double>(int, int, const LaunchArgs&, int, int);
template void launch_dirac<float>(int, const LaunchArgs&, int, int);
template void launch_dirac<double>(int, const LaunchArgs&, int, int);
template void launch_synthesis<float>(int, int, const LaunchArgs&, int, int);
template void launch_synthesis<double>(int, int, const LaunchArgs&, int, int);
template void launch_synthesis_final<float>(const LaunchArgs&, int, int, int, int);
template void launch_coarse<float>(const LaunchArgs&);
template void launch_coarse<double>(const LaunchArgs&);
template int coarse_level<float>(int, int);
template int coarse_level<double>(int, int);
template void launch_synthesis_final<double>(const LaunchArgs&, int, int, int, int);

}  // namespace psara
