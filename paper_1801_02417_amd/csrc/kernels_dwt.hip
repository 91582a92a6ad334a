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
// with c the normalised coefficient.  Intermediate low-low bands go to a per-basis
// scratch array.  Synthesis mirrors this from the coarsest level down; its last level sums
// every wavelet basis of a tile in registers and writes the image once.  The Dirac part of
// the dual update is pointwise and is fused into the primal kernel instead.
#include "common.hpp"
#include "launch.hpp"

namespace psara {

template <typename R> struct DwtTile;
// TO: analysis output tile per band; TS: synthesis output tile (levels L..2); TF: last level
template <> struct DwtTile<float> { static constexpr int TO = 16; static constexpr int TS = 32; static constexpr int TF = 16; };
template <> struct DwtTile<double> { static constexpr int TO = 8; static constexpr int TS = 16; static constexpr int TF = 16; };

template <typename R>
__device__ inline void v4_fma(V4<R>& acc, R w, const V4<R>& x) {
  acc.x += w * x.x; acc.y += w * x.y; acc.z += w * x.z; acc.w += w * x.w;
}
template <typename R>
__device__ inline V4<R> v4_zero() { V4<R> v; v.x = v.y = v.z = v.w = R(0); return v; }

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
  } else {
    k1.add((double)c.x); k1.add((double)c.y); k1.add((double)c.z); k1.add((double)c.w);
    k2.add((double)c.x * c.x); k2.add((double)c.y * c.y); k2.add((double)c.z * c.z); k2.add((double)c.w * c.w);
  }
}

template <typename R>
__device__ inline void write_partials(const ProbDesc& P, int part, const KSum& k1, const KSum& k2, int two, double* red) {
  double* gen = P.partials + 2 * (size_t)P.n_p6;
  const KSum t1 = block_reduce(k1, red);
  if (threadIdx.x == 0) { gen[2 * part] = t1.s; gen[2 * part + 1] = t1.c; }
  if (two) {
    const KSum t2 = block_reduce(k2, red);
    if (threadIdx.x == 0) { gen[2 * (part + P.gen_stride)] = t2.s; gen[2 * (part + P.gen_stride) + 1] = t2.c; }
  }
}

// ---------------------------------------------------------------------------------------------
// Analysis of level `level` (1 = finest) for every wavelet basis.
// items: {prob, wavelet index, tile, partial index}
template <typename R, int MODE>
__global__ void __launch_bounds__(256)
analysis_kernel(const ProbDesc* __restrict__ descs, const int4* __restrict__ items, int level, int src_slot, int out_coef) {
  constexpr int TO = DwtTile<R>::TO;
  constexpr int IN = 2 * TO + kMaxFilter - 2;
  __shared__ V4<R> sin_[IN * IN];
  __shared__ V4<R> rowt[IN * 2 * TO];
  __shared__ R hf[kMaxFilter], gf[kMaxFilter];
  __shared__ double red[8];
  const int4 it = items[blockIdx.x];
  const ProbDesc& P = descs[it.x];
  const int n = P.n, w = it.y;
  const int m = n >> (level - 1), h = m >> 1;
  const int to = min(TO, h), tps = h / to;
  const int o1 = (it.z / tps) * to, o2 = (it.z % tps) * to;
  const int F = P.wav_len[w];
  const int in = 2 * to + F - 2;
  if (threadIdx.x < F) {
    const R v = ((const R*)P.filters)[w * kMaxFilter + threadIdx.x];
    hf[threadIdx.x] = v;
  }
  __syncthreads();
  if (threadIdx.x < F) gf[threadIdx.x] = ((threadIdx.x & 1) ? R(-1) : R(1)) * hf[F - 1 - threadIdx.x];
  const V4<R>* __restrict__ src = (level == 1)
      ? (const V4<R>*)P.img[src_slot]
      : (const V4<R>*)P.ll + (size_t)w * P.ll_stride + P.ll_off[level - 1];
  for (int q = threadIdx.x; q < in * in; q += blockDim.x) {
    const int a = q / in, b = q - a * in;
    sin_[q] = src[(size_t)((2 * o1 + a) & (m - 1)) * m + ((2 * o2 + b) & (m - 1))];
  }
  __syncthreads();
  // rows: along the column index
  for (int q = threadIdx.x; q < in * to; q += blockDim.x) {
    const int a = q / to, k = q - a * to;
    V4<R> sa = v4_zero<R>(), sd = v4_zero<R>();
    const V4<R>* row = sin_ + a * in + 2 * k;
    for (int j = 0; j < F; ++j) { v4_fma(sa, hf[j], row[j]); v4_fma(sd, gf[j], row[j]); }
    rowt[a * (2 * to) + k] = sa;
    rowt[a * (2 * to) + to + k] = sd;
  }
  __syncthreads();
  // columns
  const size_t base = (size_t)(P.has_dirac + w) * n * n;
  const bool last = (level == P.levels);
  V4<R>* llout = (V4<R>*)P.ll + (size_t)w * P.ll_stride + P.ll_off[level];
  KSum k1, k2;
  for (int q = threadIdx.x; q < to * 2 * to; q += blockDim.x) {
    const int kr = q / (2 * to), c = q - kr * (2 * to);
    V4<R> ca = v4_zero<R>(), cd = v4_zero<R>();
    for (int j = 0; j < F; ++j) {
      const V4<R> x = rowt[(2 * kr + j) * (2 * to) + c];
      v4_fma(ca, hf[j], x);
      v4_fma(cd, gf[j], x);
    }
    const int col = (c < to) ? o2 + c : h + o2 + (c - to);
    const int rowa = o1 + kr, rowd = h + o1 + kr;
    if (c < to && !last) {
      llout[(size_t)rowa * h + col] = ca;        // low-low band feeds the next level
    } else {
      apply_coef<R, MODE>(P, out_coef, base + (size_t)rowa * n + col, ca, k1, k2);
    }
    apply_coef<R, MODE>(P, out_coef, base + (size_t)rowd * n + col, cd, k1, k2);
  }
  if (MODE == AM_OBJECTIVE || MODE == AM_MOMENTS) write_partials<R>(P, it.w, k1, k2, MODE == AM_MOMENTS, red);
}

// Dirac block for the non-dual modes.  items: {prob, block of 256 pixels, -, partial index}
template <typename R, int MODE>
__global__ void __launch_bounds__(256)
dirac_kernel(const ProbDesc* __restrict__ descs, const int4* __restrict__ items, int src_slot, int out_coef) {
  __shared__ double red[8];
  const int4 it = items[blockIdx.x];
  const ProbDesc& P = descs[it.x];
  const int N = P.n * P.n;
  const int p = it.y * 256 + threadIdx.x;
  KSum k1, k2;
  if (p < N) apply_coef<R, MODE>(P, out_coef, (size_t)p, ((const V4<R>*)P.img[src_slot])[p], k1, k2);
  if (MODE == AM_OBJECTIVE || MODE == AM_MOMENTS) write_partials<R>(P, it.w, k1, k2, MODE == AM_MOMENTS, red);
}

// ---------------------------------------------------------------------------------------------
// Synthesis, shared by the per-level kernel and the last level.  Computes one to x to tile of
// the level-(level-1) low-low band (or the image at level 1) of wavelet w into `acc`.
template <typename R>
struct SynSmem {
  static constexpr int TS = DwtTile<R>::TS;
  static constexpr int KW = TS / 2 + kMaxFilter / 2 - 1;
  V4<R> band[4][KW * KW];      // LL, HL (top-right), LH (bottom-left), HH windows
  V4<R> cola[TS * KW], cold[TS * KW];
  R hf[kMaxFilter], gf[kMaxFilter];
  double red[8];
};

template <typename R>
__device__ void synth_tile(const ProbDesc& P, SynSmem<R>& sm, int w, int level, int o1, int o2, int to,
                           int src_coef, V4<R>* acc /* per-thread outputs */, int nper) {
  const int n = P.n;
  const int m = n >> (level - 1), h = m >> 1;
  const int F = P.wav_len[w];
  const int KW = to / 2 + F / 2 - 1;
  const int ks1 = o1 / 2 - F / 2 + 1, ks2 = o2 / 2 - F / 2 + 1;
  __syncthreads();
  if (threadIdx.x < F) sm.hf[threadIdx.x] = ((const R*)P.filters)[w * kMaxFilter + threadIdx.x];
  __syncthreads();
  if (threadIdx.x < F) sm.gf[threadIdx.x] = ((threadIdx.x & 1) ? R(-1) : R(1)) * sm.hf[F - 1 - threadIdx.x];
  const V4<R>* __restrict__ A = (const V4<R>*)P.coef[src_coef] + (size_t)(P.has_dirac + w) * n * n;
  const V4<R>* __restrict__ LL = (level == P.levels) ? nullptr
      : (const V4<R>*)P.ll + (size_t)w * P.ll_stride + P.ll_off[level];
  for (int q = threadIdx.x; q < KW * KW; q += blockDim.x) {
    const int a = q / KW, b = q - a * KW;
    const int r = (ks1 + a) & (h - 1), c = (ks2 + b) & (h - 1);
    sm.band[0][q] = LL ? LL[(size_t)r * h + c] : A[(size_t)r * n + c];
    sm.band[1][q] = A[(size_t)r * n + h + c];
    sm.band[2][q] = A[(size_t)(h + r) * n + c];
    sm.band[3][q] = A[(size_t)(h + r) * n + h + c];
  }
  __syncthreads();
  // inverse column transform (along the row index): rows at full resolution
  for (int q = threadIdx.x; q < to * KW; q += blockDim.x) {
    const int ir = q / KW, b = q - ir * KW;
    const int i = o1 + ir;
    V4<R> sa = v4_zero<R>(), sd = v4_zero<R>();
    for (int j = (i & 1); j < F; j += 2) {
      const int a = ((i - j) >> 1) - ks1;
      v4_fma(sa, sm.hf[j], sm.band[0][a * KW + b]);
      v4_fma(sa, sm.gf[j], sm.band[2][a * KW + b]);
      v4_fma(sd, sm.hf[j], sm.band[1][a * KW + b]);
      v4_fma(sd, sm.gf[j], sm.band[3][a * KW + b]);
    }
    sm.cola[ir * KW + b] = sa;
    sm.cold[ir * KW + b] = sd;
  }
  __syncthreads();
  // inverse row transform (along the column index)
  for (int t = 0; t < nper; ++t) {
    const int q = threadIdx.x + t * blockDim.x;
    if (q >= to * to) break;
    const int ir = q / to, ic = q - ir * to;
    const int i = o2 + ic;
    V4<R> s = acc[t];
    for (int j = (i & 1); j < F; j += 2) {
      const int b = ((i - j) >> 1) - ks2;
      v4_fma(s, sm.hf[j], sm.cola[ir * KW + b]);
      v4_fma(s, sm.gf[j], sm.cold[ir * KW + b]);
    }
    acc[t] = s;
  }
}

// Levels L..2: items {prob, wavelet index, tile, -}; writes the low-low band of level-1.
template <typename R>
__global__ void __launch_bounds__(256)
synthesis_kernel(const ProbDesc* __restrict__ descs, const int4* __restrict__ items, int level, int src_coef) {
  __shared__ SynSmem<R> sm;
  constexpr int TS = DwtTile<R>::TS;
  constexpr int NPER = (TS * TS + 255) / 256;
  const int4 it = items[blockIdx.x];
  const ProbDesc& P = descs[it.x];
  const int w = it.y;
  const int m = P.n >> (level - 1);
  const int to = min(TS, m), tps = m / to;
  const int o1 = (it.z / tps) * to, o2 = (it.z % tps) * to;
  V4<R> acc[NPER];
#pragma unroll
  for (int t = 0; t < NPER; ++t) acc[t] = v4_zero<R>();
  synth_tile<R>(P, sm, w, level, o1, o2, to, src_coef, acc, NPER);
  V4<R>* out = (V4<R>*)P.ll + (size_t)w * P.ll_stride + P.ll_off[level - 1];
#pragma unroll
  for (int t = 0; t < NPER; ++t) {
    const int q = threadIdx.x + t * blockDim.x;
    if (q < to * to) out[(size_t)(o1 + q / to) * m + o2 + q % to] = acc[t];
  }
}

// Level 1 of every wavelet basis, summed, times 1/sqrt(nb); optionally plus the Dirac block.
// items: {prob, tile, -, -}
template <typename R>
__global__ void __launch_bounds__(256)
synthesis_final_kernel(const ProbDesc* __restrict__ descs, const int4* __restrict__ items, int src_coef, int dst_slot, int add_dirac) {
  __shared__ SynSmem<R> sm;
  constexpr int TS = DwtTile<R>::TF;
  constexpr int NPER = (TS * TS + 255) / 256;
  const int4 it = items[blockIdx.x];
  const ProbDesc& P = descs[it.x];
  const int n = P.n;
  const int to = min(TS, n), tps = n / to;
  const int o1 = (it.y / tps) * to, o2 = (it.y % tps) * to;
  V4<R> acc[NPER];
#pragma unroll
  for (int t = 0; t < NPER; ++t) acc[t] = v4_zero<R>();
  for (int w = 0; w < P.nwav; ++w) synth_tile<R>(P, sm, w, 1, o1, o2, to, src_coef, acc, NPER);
  const R nm = R(P.norm);
  const V4<R>* dirac = (const V4<R>*)P.coef[src_coef];
  V4<R>* out = (V4<R>*)P.img[dst_slot];
#pragma unroll
  for (int t = 0; t < NPER; ++t) {
    const int q = threadIdx.x + t * blockDim.x;
    if (q < to * to) {
      const size_t idx = (size_t)(o1 + q / to) * n + o2 + q % to;
      V4<R> s = acc[t];
      if (add_dirac && P.has_dirac) {
        const V4<R> d = dirac[idx];
        s.x += d.x; s.y += d.y; s.z += d.z; s.w += d.w;
      }
      s.x *= nm; s.y *= nm; s.z *= nm; s.w *= nm;
      out[idx] = s;
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Coarse levels c..L of one wavelet basis in a single workgroup: the low-low band entering
// level c (at most CoarseMax<R> on a side) is held in LDS; analysis runs level by level with
// the dual update of every coefficient, then synthesis runs back from level L to level c on
// the updated duals and leaves the low-low band of level c-1 in the level scratch, where the
// next synthesis launch reads it.  Replaces 2 (L - c + 1) small launches by one.
// items: {prob, wavelet index, -, -}
template <typename R> struct CoarseMax { static constexpr int value = sizeof(R) == 4 ? 64 : 32; };

template <typename R>
__global__ void __launch_bounds__(1024)
coarse_kernel(const ProbDesc* __restrict__ descs, const int4* __restrict__ items, int c_level) {
  constexpr int MM = CoarseMax<R>::value;
  __shared__ V4<R> bufA[MM * MM];
  __shared__ V4<R> bufB[MM * MM];
  __shared__ R hf[kMaxFilter], gf[kMaxFilter];
  const int4 it = items[blockIdx.x];
  const ProbDesc& P = descs[it.x];
  const int n = P.n, w = it.y, L = P.levels;
  const int F = P.wav_len[w];
  const int nt = blockDim.x;
  if (threadIdx.x < F) hf[threadIdx.x] = ((const R*)P.filters)[w * kMaxFilter + threadIdx.x];
  __syncthreads();
  if (threadIdx.x < F) gf[threadIdx.x] = ((threadIdx.x & 1) ? R(-1) : R(1)) * hf[F - 1 - threadIdx.x];
  V4<R>* __restrict__ ll = (V4<R>*)P.ll + (size_t)w * P.ll_stride;
  V4<R>* __restrict__ A = (V4<R>*)P.coef[COEF_A];
  const V4<R>* __restrict__ GW = (const V4<R>*)P.coef[COEF_GW];
  const size_t base = (size_t)(P.has_dirac + w) * n * n;
  const R nm = R(P.norm), r1 = R(P.rho1);
  int m = n >> (c_level - 1);
  for (int q = threadIdx.x; q < m * m; q += nt) bufA[q] = ll[P.ll_off[c_level - 1] + q];
  __syncthreads();
  auto dual = [&](size_t idx, const V4<R>& raw) {
    const V4<R> g = GW[idx];
    V4<R> a = A[idx];
    a.x = fmin(fmax(a.x + r1 * nm * raw.x, -g.x), g.x);
    a.y = fmin(fmax(a.y + r1 * nm * raw.y, -g.y), g.y);
    a.z = fmin(fmax(a.z + r1 * nm * raw.z, -g.z), g.z);
    a.w = fmin(fmax(a.w + r1 * nm * raw.w, -g.w), g.w);
    A[idx] = a;
  };
  // ---- analysis c..L (bufA holds the m x m low-low band) ----
  for (int l = c_level; l <= L; ++l) {
    const int h = m >> 1;
    for (int q = threadIdx.x; q < m * m; q += nt) {          // rows: bufB[r][k] = a, bufB[r][h+k] = d
      const int r = q / m, k = q - r * m;
      const int kk = k < h ? k : k - h;
      const R* flt = k < h ? hf : gf;
      V4<R> acc = v4_zero<R>();
      for (int j = 0; j < F; ++j) v4_fma(acc, flt[j], bufA[r * m + ((2 * kk + j) & (m - 1))]);
      bufB[q] = acc;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < m * m; q += nt) {          // columns
      const int k1 = q / m, col = q - k1 * m;
      const int kk = k1 < h ? k1 : k1 - h;
      const R* flt = k1 < h ? hf : gf;
      V4<R> acc = v4_zero<R>();
      for (int j = 0; j < F; ++j) v4_fma(acc, flt[j], bufB[((2 * kk + j) & (m - 1)) * m + col]);
      if (k1 < h && col < h && l < L) bufA[k1 * h + col] = acc;     // next level's input
      else dual(base + (size_t)k1 * n + col, acc);
    }
    __syncthreads();
    m = h;
  }
  __threadfence_block();
  __syncthreads();
  // ---- synthesis L..c on the updated duals (bufA: the h x h low-low input) ----
  const V4<R>* __restrict__ Ac = A;
  {
    const int h = n >> L;
    for (int q = threadIdx.x; q < h * h; q += nt) bufA[q] = Ac[base + (size_t)(q / h) * n + q % h];
  }
  __syncthreads();
  for (int l = L; l >= c_level; --l) {
    const int mo = n >> (l - 1), h = mo >> 1;
    // inverse column transform: bufB[ir][b] (ir < mo, b < h) from LL/LH, bufB[mo*h + ...] from HL/HH
    for (int q = threadIdx.x; q < mo * h; q += nt) {
      const int ir = q / h, b = q - ir * h;
      V4<R> sa = v4_zero<R>(), sd = v4_zero<R>();
      for (int j = (ir & 1); j < F; j += 2) {
        const int r = ((ir - j) >> 1) & (h - 1);
        v4_fma(sa, hf[j], bufA[r * h + b]);
        v4_fma(sa, gf[j], Ac[base + (size_t)(h + r) * n + b]);
        v4_fma(sd, hf[j], Ac[base + (size_t)r * n + h + b]);
        v4_fma(sd, gf[j], Ac[base + (size_t)(h + r) * n + h + b]);
      }
      bufB[q] = sa;
      bufB[mo * h + q] = sd;
    }
    __syncthreads();
    // inverse row transform into bufA (mo x mo)
    for (int q = threadIdx.x; q < mo * mo; q += nt) {
      const int ir = q / mo, ic = q - ir * mo;
      V4<R> s = v4_zero<R>();
      for (int j = (ic & 1); j < F; j += 2) {
        const int b = ((ic - j) >> 1) & (h - 1);
        v4_fma(s, hf[j], bufB[ir * h + b]);
        v4_fma(s, gf[j], bufB[mo * h + ir * h + b]);
      }
      bufA[q] = s;
    }
    __syncthreads();
  }
  const int mo = n >> (c_level - 1);
  for (int q = threadIdx.x; q < mo * mo; q += nt) ll[P.ll_off[c_level - 1] + q] = bufA[q];
}

template <typename R>
int coarse_level(int n, int levels) {
  // first level >= 2 whose input low-low band fits the LDS buffers
  for (int c = 2; c <= levels; ++c)
    if ((n >> (c - 1)) <= CoarseMax<R>::value) return c;
  return levels + 1;
}

template <typename R>
void launch_coarse(const LaunchArgs& a, int c_level) {
  if (a.nitems <= 0) return;
  hipLaunchKernelGGL((coarse_kernel<R>), dim3(a.nitems), dim3(1024), 0, a.stream, a.descs, a.items, c_level);
}

template <typename R>
void launch_analysis(int mode, int level, const LaunchArgs& a, int src_slot, int out_coef) {
  if (a.nitems <= 0) return;
  const dim3 g(a.nitems), b(256);
  switch (mode) {
    case AM_DUAL: hipLaunchKernelGGL((analysis_kernel<R, AM_DUAL>), g, b, 0, a.stream, a.descs, a.items, level, src_slot, out_coef); break;
    case AM_STORE: hipLaunchKernelGGL((analysis_kernel<R, AM_STORE>), g, b, 0, a.stream, a.descs, a.items, level, src_slot, out_coef); break;
    case AM_REWEIGHT: hipLaunchKernelGGL((analysis_kernel<R, AM_REWEIGHT>), g, b, 0, a.stream, a.descs, a.items, level, src_slot, out_coef); break;
    case AM_OBJECTIVE: hipLaunchKernelGGL((analysis_kernel<R, AM_OBJECTIVE>), g, b, 0, a.stream, a.descs, a.items, level, src_slot, out_coef); break;
    default: hipLaunchKernelGGL((analysis_kernel<R, AM_MOMENTS>), g, b, 0, a.stream, a.descs, a.items, level, src_slot, out_coef); break;
  }
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
    default: hipLaunchKernelGGL((dirac_kernel<R, AM_DUAL>), g, b, 0, a.stream, a.descs, a.items, src_slot, out_coef); break;
  }
}

template <typename R>
void launch_synthesis(int level, int /*coarsest*/, const LaunchArgs& a, int src_coef, int /*dst_slot*/) {
  if (a.nitems <= 0) return;
  hipLaunchKernelGGL((synthesis_kernel<R>), dim3(a.nitems), dim3(256), 0, a.stream, a.descs, a.items, level, src_coef);
}

template <typename R>
void launch_synthesis_final(const LaunchArgs& a, int src_coef, int dst_slot, int add_dirac) {
  if (a.nitems <= 0) return;
  hipLaunchKernelGGL((synthesis_final_kernel<R>), dim3(a.nitems), dim3(256), 0, a.stream, a.descs, a.items, src_coef, dst_slot, add_dirac);
}

template void launch_analysis<float>(int, int, const LaunchArgs&, int, int);
template void launch_analysis<double>(int, int, const LaunchArgs&, int, int);
template void launch_dirac<float>(int, const LaunchArgs&, int, int);
template void launch_dirac<double>(int, const LaunchArgs&, int, int);
template void launch_synthesis<float>(int, int, const LaunchArgs&, int, int);
template void launch_synthesis<double>(int, int, const LaunchArgs&, int, int);
template void launch_synthesis_final<float>(const LaunchArgs&, int, int, int);
template void launch_coarse<float>(const LaunchArgs&, int);
template void launch_coarse<double>(const LaunchArgs&, int);
template int coarse_level<float>(int, int);
template int coarse_level<double>(int, int);
template void launch_synthesis_final<double>(const LaunchArgs&, int, int, int);

}  // namespace psara
