// Oversampled-grid FFT passes of the measurement operator (Sec. 4.1, eq. meas_op:
// F and its adjoint, fused with the zero-padding / scaling Z and the crop / real part).
//
// The 2-D transform of a K x K grid (K = 2n) is split in two line passes through an
// intermediate `half` array of K x n cells stored transposed, [k2][r]:
//   forward  P4: image row r (n pixels, scaled, placed at wrapped positions) -> FFT along
//                columns -> half[k2][r]
//            P5: half[k2][:] (n nonzero rows at wrapped positions) -> FFT along rows ->
//                grid[k2][k1]
//   adjoint  P8: grid[k2][:] -> inverse FFT along rows -> keep the n cropped rows ->
//                half[k2][r]
//            P9: half[:][r] -> inverse FFT along columns -> keep the n cropped columns,
//                real part, scaling -> image row r
// so the zero half of the padded image is never read and the crop never writes unused
// cells.  The grid is stored transposed ([k2][k1]); the de-gridding and gridding kernels
// index it that way.  Every cell carries the four Stokes channels, which share twiddles.
//
// Line FFTs run in LDS as Stockham autosort passes (radix 8, then 4 or 2) with the data of
// each butterfly held in registers across a barrier, so a single LDS buffer suffices.  Each
// thread owns one Stokes channel of 8 cells per pass (one radix-8, two radix-4 or four
// radix-2 butterflies).
#include "common.hpp"
#include "launch.hpp"
#include "primal.hpp"

namespace psara {

template <typename R>
__device__ inline void dft2(cplx<R>& a, cplx<R>& b) {
  cplx<R> t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

// multiply by -i (forward) or +i (inverse)
template <typename R>
__device__ inline cplx<R> rot(cplx<R> a, bool inv) { return inv ? cmk(-a.im, a.re) : cmk(a.im, -a.re); }

template <typename R>
__device__ inline void dft4(cplx<R>& a0, cplx<R>& a1, cplx<R>& a2, cplx<R>& a3, bool inv) {
  cplx<R> t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = rot(csub(a1, a3), inv);
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

template <typename R>
__device__ inline void dft8(cplx<R>* a, bool inv) {
  cplx<R> e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  cplx<R> o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
  dft4(e0, e1, e2, e3, inv);
  dft4(o0, o1, o2, o3, inv);
  const R h = R(0.70710678118654752440084436210485);
  // o_k *= w8^k, w8 = exp(-+ 2 pi i / 8)
  o1 = inv ? cmk(h * (o1.re - o1.im), h * (o1.re + o1.im)) : cmk(h * (o1.re + o1.im), h * (o1.im - o1.re));
  o2 = rot(o2, inv);
  o3 = inv ? cmk(-h * (o3.re + o3.im), h * (o3.re - o3.im)) : cmk(h * (o3.im - o3.re), -h * (o3.re + o3.im));
  a[0] = cadd(e0, o0); a[4] = csub(e0, o0);
  a[1] = cadd(e1, o1); a[5] = csub(e1, o1);
  a[2] = cadd(e2, o2); a[6] = csub(e2, o2);
  a[3] = cadd(e3, o3); a[7] = csub(e3, o3);
}

// One Stockham pass of radix RAD over the lines in LDS.  A thread owns one Stokes channel
// `ch` of 8 cells: it reads the inputs of its 8/RAD butterflies into registers and writes
// the outputs after a barrier, so the pass is done in place.  The four lanes of a cell are
// adjacent, so their 8-byte (16-byte in FP64) accesses are contiguous.
template <typename R, int RAD>
__device__ inline void stockham_pass(cplx<R>* x, int K, int Ns, int tl, int per_line, int ch, bool inv,
                                     const cplx<R>* __restrict__ tw) {
  constexpr int NB = 8 / RAD;
  constexpr int LR = RAD == 8 ? 3 : RAD == 4 ? 2 : 1;   // log2 RAD
  // K and Ns are powers of two: divisions by them are shifts and masks
  const int lk = lg2(K), ls = lg2(Ns);
  const int stride = K >> LR;
  cplx<R> v[8];
  // the pass's twiddles first, so that their loads are in flight across the barrier
  const int twstep = K >> (ls + LR);
  cplx<R> wt[NB][RAD];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int k = (tl + b * per_line) & (Ns - 1);
#pragma unroll
    for (int r = 1; r < RAD; ++r) wt[b][r] = tw[r * k * twstep];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int b = q / RAD, r = q - b * RAD;
    v[q] = x[4 * (tl + b * per_line + r * stride) + ch];
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = tl + b * per_line;
    const int k = j & (Ns - 1);
#pragma unroll
    for (int r = 1; r < RAD; ++r) {
      cplx<R> w = wt[b][r];
      if (inv) w.im = -w.im;
      v[b * RAD + r] = cmul(v[b * RAD + r], w);
    }
    if (RAD == 8) dft8(v + b * 8, inv);
    else if (RAD == 4) dft4(v[b * 4], v[b * 4 + 1], v[b * 4 + 2], v[b * 4 + 3], inv);
    else dft2(v[b * 2], v[b * 2 + 1]);
    const int base = ((j >> ls) << (ls + LR)) + k;
#pragma unroll
    for (int r = 0; r < RAD; ++r) x[4 * (base + r * Ns) + ch] = v[b * RAD + r];
  }
}

// In-place Stockham FFT (radix 8 passes, then one radix-4 or radix-2 pass) of the lines held
// in `lds` (line l at lds + l*K).  Called by CELLS/2 threads: thread t handles channel t % 4 of
// the 8 cells of butterfly group t / 4, on line (t / 4) / (K/8).
template <typename R, int CELLS>
__device__ void fft_lines(Cell<R>* lds, int K, bool inv, const cplx<R>* __restrict__ tw) {
  const int per_line = K >> 3;
  const int ch = threadIdx.x & 3, grp = threadIdx.x >> 2;
  const int l = grp >> lg2(per_line), tl = grp & (per_line - 1);
  cplx<R>* x = (cplx<R>*)(lds + l * K);
  int Ns = 1;
  while (Ns < K) {
    const int rem = K >> lg2(Ns);
    if (rem % 8 == 0) { stockham_pass<R, 8>(x, K, Ns, tl, per_line, ch, inv, tw); Ns *= 8; }
    else if (rem % 4 == 0) { stockham_pass<R, 4>(x, K, Ns, tl, per_line, ch, inv, tw); Ns *= 4; }
    else { stockham_pass<R, 2>(x, K, Ns, tl, per_line, ch, inv, tw); Ns *= 2; }
  }
  __syncthreads();
}

// a product that is rounded on its own (never contracted into a following add)
template <typename R>
__device__ __forceinline__ R mul_rn(R a, R b) {
#pragma clang fp contract(off)
  return a * b;
}

template <typename R>
__device__ inline Cell<R> zero_cell() {
  Cell<R> c;
#pragma unroll
  for (int s = 0; s < 4; ++s) c.s[s] = cmk(R(0), R(0));
  return c;
}

// PASS: 0 = P4 image rows -> half, 1 = P5 half -> grid, 2 = P8 grid -> half, 3 = P9 half -> image,
// 4 = P9, P1 and P4 of the next iteration in one pass: half -> inverse row FFT -> Re phi^dagger B
// of the row's pixels (kept in LDS) -> primal step -> X -> forward row FFT -> half.
// PM >= 0 (PASS 0 and 4): the primal step of mode PM runs on each pixel as the row is loaded
// and the row FFT takes the X it returns (P1 fused into P4).
// items: {prob, first line, -, -}; CELLS/K lines per workgroup.  The row passes (P4, P9) use
// several lines per workgroup so that their transposed accesses to `half` cover whole cache
// lines (four consecutive image rows per k2 in FP32).
template <typename R, int CELLS, int PASS, int PM = -1>
__global__ void __launch_bounds__(CELLS / 2)
fft_pass_kernel(const ProbDesc* __restrict__ descs, const int4* __restrict__ items, int src_slot, int dst_slot) {
  __shared__ Cell<R> lds[CELLS];
  const int4 it = items[blockIdx.x];
  const ProbDesc& P = descs[it.x];
  if (halted(P)) return;                 // stopped by an adaptive run
  const int n = P.n, K = P.K, h2 = n / 2;
  const int lines = CELLS / K;
  const int lgK = lg2(K), lgL = lg2(lines), lgN = lg2(n);   // all powers of two
  const int line0 = it.y;
  const R* __restrict__ s = (const R*)P.deapod;
  Cell<R>* __restrict__ half = (Cell<R>*)P.half;
  Cell<R>* __restrict__ grid = (Cell<R>*)P.grid;
  const int nthr = CELLS / 2;

  // the partial-slot table and the slot-box unions of the gridding tiles this workgroup's lines
  // read (their tile rows and the rows before them), staged once so the per-cell gathers index LDS
  constexpr int kTslMax = CELLS / 256 + 2048 / 8;
  __shared__ int2 tsl[PASS == 2 ? kTslMax : 1];
  __shared__ int tbx[PASS == 2 ? kTslMax : 1];
  __shared__ double red[PASS == 2 ? 2 * ((CELLS / 2 + 63) / 64) : 1];
  int trow0 = 0;
  R gfac = R(1);
  if (PASS == 2) {
    // the factor of the gridded values (src_slot: 0 the one the grid pass stored; 1 the l2-ball
    // factor c = rho2 max(0, 1 - epsilon / ||Bv||) from the fused pass's per-chunk partials,
    // reduced by every workgroup in the same fixed order and stored, with ||Bv||^2, by the
    // problem's first; 2 one)
    if (src_slot == 1) {
      const double v2 = block_sum_partials(chunk_partials(P), P.n_slots, red);
      const double vn = sqrt(v2);
      const double c = (vn > P.eps) ? P.rho2 * (1.0 - P.eps / vn) : 0.0;
      if (line0 == 0 && threadIdx.x == 0) {
        P.scal[SC_CFAC] = c;
        P.scal[SC_VNORM2] = v2;
        P.scal[SC_GFAC] = c;
      }
      gfac = R(c);
    } else if (src_slot == 0) {
      gfac = R(P.scal[SC_GFAC]);
    }
    const int ntg = P.ntile_side_g;
    trow0 = line0 / kGridTile - 1;
    const int ntr = min(K - 1, line0 + lines - 1) / kGridTile - trow0 + 1;
    for (int i = threadIdx.x; i < ntr * ntg; i += nthr) {
      const int rr = i >> lg2(ntg), u1 = i & (ntg - 1);
      const int t = u1 * ntg + ((trow0 + rr + ntg) & (ntg - 1));
      const int2 sl = P.tile_slots[t];
      const int bx = P.tile_box[t];
      tsl[i] = sl;
      tbx[i] = bx;
    }
    __syncthreads();
  }
  // P9 + P1 + P4: the primal step's inputs of this thread's pixels (its cells q and q + nthr in
  // the crop) are requested now, so their loads overlap the loads and the inverse FFT below
  // (not with 1024 threads, whose 128 registers would spill them)
  constexpr bool kPrefetch = PASS == 4 && PM >= 0 && CELLS <= 1024;
  PrimalIn<R> pin[kPrefetch ? 2 : 1];
  if constexpr (kPrefetch) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int q = threadIdx.x + u * nthr;
      const int l = q >> lgK, k = q & (K - 1), r = line0 + l;
      const int col = (k < h2) ? k + h2 : ((k >= K - h2) ? k - (K - h2) : -1);
      if (r < n && col >= 0) pin[u] = primal_load<R, (PM < 0 ? 0 : PM)>(P, r * n + col);
    }
  }
  // ---- load ----
  // (the FP64 kernel with 1024 threads, 128 registers, keeps the gather one pair at a time: the
  // eight pairs' cells in flight would spill)
  constexpr bool kRounds = PASS == 2 && !(sizeof(R) == 8 && CELLS > 1024);
  if constexpr (kRounds) {
    // the gridded values of the thread's cells q and q + nthr: the partial slots of each cell's
    // tile and of the tiles whose halos reach it (the previous tile in k1, in k2, and in both),
    // times the factor the gridding pass left out.  Each (cell, tile) pair's first slot cell and
    // slot count come from the staged tables; the slots are then added round by round (slot
    // index sl of every pair, pairs in a fixed order), and a round loads all eight pairs' cells
    // before adding any (a pair with fewer slots, or none, loads a cell of an existing slot that
    // it does not add), so those loads are in flight together
    const int ntg = P.ntile_side_g, RG = kGridTile + P.T - 1;
    const Cell<R>* __restrict__ gp = (const Cell<R>*)P.gpart;
    const Cell<R>* src[2][4];
    int cnt[2][4];
    int rounds = 0;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int q = threadIdx.x + u * nthr;
      const int l = q >> lgK, k = q & (K - 1), k2 = line0 + l;
      const int t1 = k / kGridTile, t2 = k2 / kGridTile, a1 = k - t1 * kGridTile, a2 = k2 - t2 * kGridTile;
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        const int d1 = d & 1, d2 = d >> 1;
        const int o1 = a1 + d1 * kGridTile, o2 = a2 + d2 * kGridTile;
        src[u][d] = gp;
        cnt[u][d] = 0;
        if (k2 >= K || o1 >= RG || o2 >= RG) continue;
        const int ti = (t2 - d2 - trow0) * ntg + ((t1 - d1 + ntg) & (ntg - 1));
        if (!in_box(tbx[ti], o1, o2)) continue;          // no slot of the tile reaches it
        const int2 ts = tsl[ti];
        src[u][d] = gp + (size_t)ts.x * RG * RG + o2 * RG + o1;
        cnt[u][d] = ts.y;
        rounds = max(rounds, ts.y);
      }
    }
    Cell<R> c[2] = {zero_cell<R>(), zero_cell<R>()};
    for (int sl = 0; sl < rounds; ++sl) {
      Cell<R> o[2][4];
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int d = 0; d < 4; ++d) o[u][d] = src[u][d][sl < cnt[u][d] ? (size_t)sl * RG * RG : 0];
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int d = 0; d < 4; ++d)
          if (sl < cnt[u][d]) {
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) c[u].s[ch] = cadd(c[u].s[ch], o[u][d].s[ch]);
          }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) { c[u].s[ch].re *= gfac; c[u].s[ch].im *= gfac; }
      lds[threadIdx.x + u * nthr] = c[u];
    }
  }
  if constexpr (PASS == 1 || PASS >= 3) {
    // both of the thread's cells are loaded before either is stored, so the two loads are in
    // flight together (P5 reads half[k2][r] into line order; P9 and the fused row pass read it
    // transposed into their rows)
    Cell<R> cv[2];
    int dst[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int q = threadIdx.x + u * nthr;
      cv[u] = zero_cell<R>();
      if constexpr (PASS == 1) {
        const int l = q >> lgK, k = q & (K - 1), k2 = line0 + l;
        const int r = (k < h2) ? k + h2 : ((k >= K - h2) ? k - (K - h2) : -1);
        if (k2 < K && r >= 0) cv[u] = half[(size_t)k2 * n + r];
        dst[u] = q;
      } else {
        const int k2 = q >> lgL, l = q & (lines - 1), r = line0 + l;
        if (r < n) cv[u] = half[(size_t)k2 * n + r];
        dst[u] = l * K + k2;
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) lds[dst[u]] = cv[u];
  }
  // P4 (the rows of X, or with PM the primal step's X, staged as they are computed), and P8's
  // gathers one (cell, tile) pair at a time where the rounds above would spill
  if constexpr (PASS == 0 || (PASS == 2 && !kRounds)) {
  for (int q = threadIdx.x; q < lines * K; q += nthr) {
    Cell<R> c = zero_cell<R>();
    if (PASS == 0) {
      const int l = q >> lgK, k = q & (K - 1), r = line0 + l;
      const int col = (k < h2) ? k + h2 : ((k >= K - h2) ? k - (K - h2) : -1);
      if (r < n && col >= 0) {
        V4<R> v;
        if (PM >= 0) v = primal_pixel<R, (PM < 0 ? 0 : PM)>(P, r * n + col);
        else v = ((const V4<R>*)P.img[src_slot])[(size_t)r * n + col];
        const R sc = s[r] * s[col];
        c.s[0].re = v.x * sc; c.s[1].re = v.y * sc; c.s[2].re = v.z * sc; c.s[3].re = v.w * sc;
      }
      lds[q] = c;
    } else {
      // the gathers one (cell, tile) pair at a time, in the order of the rounds above
      const int l = q >> lgK, k = q & (K - 1), k2 = line0 + l;
      if (k2 < K) {
        const int ntg = P.ntile_side_g, RG = kGridTile + P.T - 1;
        const int t1 = k / kGridTile, t2 = k2 / kGridTile, a1 = k - t1 * kGridTile, a2 = k2 - t2 * kGridTile;
        const Cell<R>* src[4];
        int cnt[4], rounds = 0;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          const int d1 = d & 1, d2 = d >> 1;
          const int o1 = a1 + d1 * kGridTile, o2 = a2 + d2 * kGridTile;
          src[d] = (const Cell<R>*)P.gpart;
          cnt[d] = 0;
          if (o1 >= RG || o2 >= RG) continue;
          const int ti = (t2 - d2 - trow0) * ntg + ((t1 - d1 + ntg) & (ntg - 1));
          if (!in_box(tbx[ti], o1, o2)) continue;
          const int2 ts = tsl[ti];
          src[d] = (const Cell<R>*)P.gpart + (size_t)ts.x * RG * RG + o2 * RG + o1;
          cnt[d] = ts.y;
          rounds = max(rounds, ts.y);
        }
        for (int sl = 0; sl < rounds; ++sl)
#pragma unroll
          for (int d = 0; d < 4; ++d)
            if (sl < cnt[d]) {
              const Cell<R> o = src[d][(size_t)sl * RG * RG];
#pragma unroll
              for (int ch = 0; ch < 4; ++ch) c.s[ch] = cadd(c.s[ch], o.s[ch]);
            }
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) { c.s[ch].re *= gfac; c.s[ch].im *= gfac; }
      }
      lds[q] = c;
    }
  }
  }
  __syncthreads();
  // lines * K == CELLS (K divides CELLS), so every thread owns one channel of 8 cells
  fft_lines<R, CELLS>(lds, K, PASS >= 2, (const cplx<R>*)P.twiddle);

  if constexpr (PASS == 4) {
    // crop, Z^dagger and Re give Re phi^dagger B at the row's pixels; the primal step takes it
    // and its X, deapodised and zero-padded, replaces the row in place (a pixel's crop position
    // and its zero-padding position are the same cell)
    static_assert(CELLS == 2 * (CELLS / 2), "two cells per thread");
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int q = threadIdx.x + u * nthr;
      const int l = q >> lgK, k = q & (K - 1), r = line0 + l;
      const int col = (k < h2) ? k + h2 : ((k >= K - h2) ? k - (K - h2) : -1);
      Cell<R> c = zero_cell<R>();
      if (r < n && col >= 0) {
        const Cell<R> v = lds[q];
        const R sc = s[r] * s[col];
        // rounded products, not contracted into the primal step's sums: the result is bitwise
        // the one of the separate passes, which store Re phi^dagger B and read it back
        V4<R> g;
        g.x = mul_rn(v.s[0].re, sc); g.y = mul_rn(v.s[1].re, sc);
        g.z = mul_rn(v.s[2].re, sc); g.w = mul_rn(v.s[3].re, sc);
        constexpr int PMM = PM < 0 ? 0 : PM;
        const V4<R> x = kPrefetch ? primal_pixel_in<R, PMM>(P, r * n + col, g, pin[kPrefetch ? u : 0])
                                  : primal_pixel_g<R, PMM>(P, r * n + col, g);
        c.s[0].re = x.x * sc; c.s[1].re = x.y * sc; c.s[2].re = x.z * sc; c.s[3].re = x.w * sc;
      }
      lds[q] = c;
    }
    __syncthreads();
    fft_lines<R, CELLS>(lds, K, false, (const cplx<R>*)P.twiddle);
  }

  // ---- store ----
  if (PASS == 0 || PASS == 4) {
    for (int q = threadIdx.x; q < lines * K; q += nthr) {
      const int k2 = q >> lgL, l = q & (lines - 1), r = line0 + l;
      if (r < n) half[(size_t)k2 * n + r] = lds[l * K + k2];
    }
  } else if (PASS == 1) {
    for (int q = threadIdx.x; q < lines * K; q += nthr) {
      const int l = q >> lgK, k1 = q & (K - 1), k2 = line0 + l;
      if (k2 < K) grid[(size_t)k2 * K + k1] = lds[q];
    }
  } else if (PASS == 2) {
    for (int q = threadIdx.x; q < lines * n; q += nthr) {
      const int l = q >> lgN, r = q & (n - 1), k2 = line0 + l;
      const int pos = r < h2 ? r + (K - h2) : r - h2;        // (r - n/2) mod K
      if (k2 < K) half[(size_t)k2 * n + r] = lds[l * K + pos];
    }
  } else {
    V4<R>* __restrict__ out = (V4<R>*)P.img[dst_slot];
    for (int q = threadIdx.x; q < lines * n; q += nthr) {
      const int l = q >> lgN, c = q & (n - 1), r = line0 + l;
      const int pos = c < h2 ? c + (K - h2) : c - h2;
      if (r < n) {
        const Cell<R> v = lds[l * K + pos];
        const R sc = s[r] * s[c];
        V4<R> o;
        o.x = v.s[0].re * sc; o.y = v.s[1].re * sc; o.z = v.s[2].re * sc; o.w = v.s[3].re * sc;
        out[(size_t)r * n + c] = o;
      }
    }
  }
}

// the primal-step modes of the row passes (PASS 0 and 4), for one CELLS
template <typename R, int CELLS, int PASS>
void launch_row_primal_t(int mode, const LaunchArgs& a) {
  const dim3 grid(a.nitems);
#define PSARA_RP(PM) \
  hipLaunchKernelGGL((fft_pass_kernel<R, CELLS, PASS, PM>), grid, dim3(CELLS / 2), 0, a.stream, a.descs, a.items, 0, 0)
  switch (mode) {
    case PM_CONSTRAINED: PSARA_RP(PM_CONSTRAINED); break;
    case PM_INIT: PSARA_RP(PM_INIT); break;
    case PM_UNCONSTRAINED: PSARA_RP(PM_UNCONSTRAINED); break;
    case PM_TV_CONSTRAINED: PSARA_RP(PM_TV_CONSTRAINED); break;
    default: PSARA_RP(PM_TV_UNCONSTRAINED); break;
  }
#undef PSARA_RP
}

template <typename R, int PASS>
void launch_row_primal(int mode, const LaunchArgs& a, int cells) {
  if (a.nitems <= 0) return;
  if (cells == 512) launch_row_primal_t<R, 512, PASS>(mode, a);
  else if (cells == 2048) launch_row_primal_t<R, 2048, PASS>(mode, a);
  else launch_row_primal_t<R, 1024, PASS>(mode, a);
}

template <typename R>
void launch_primal_fft(int mode, const LaunchArgs& a, int cells) { launch_row_primal<R, 0>(mode, a, cells); }

template <typename R>
void launch_fused_rows(int mode, const LaunchArgs& a, int cells) { launch_row_primal<R, 4>(mode, a, cells); }

template <typename R>
void launch_fft(int pass, const LaunchArgs& a, int cells, int src_slot, int dst_slot) {
  if (a.nitems <= 0) return;
  const dim3 grid(a.nitems);
#define PSARA_FFT(C, PS) \
  hipLaunchKernelGGL((fft_pass_kernel<R, C, PS>), grid, dim3(C / 2), 0, a.stream, a.descs, a.items, src_slot, dst_slot)
  if (cells == 512) {
    switch (pass) {
      case 0: PSARA_FFT(512, 0); break;
      case 1: PSARA_FFT(512, 1); break;
      case 2: PSARA_FFT(512, 2); break;
      default: PSARA_FFT(512, 3); break;
    }
  } else if (cells == 2048) {
    switch (pass) {
      case 0: PSARA_FFT(2048, 0); break;
      case 1: PSARA_FFT(2048, 1); break;
      case 2: PSARA_FFT(2048, 2); break;
      default: PSARA_FFT(2048, 3); break;
    }
  } else {
    switch (pass) {
      case 0: PSARA_FFT(1024, 0); break;
      case 1: PSARA_FFT(1024, 1); break;
      case 2: PSARA_FFT(1024, 2); break;
      default: PSARA_FFT(1024, 3); break;
    }
  }
#undef PSARA_FFT
}

template void launch_fft<float>(int, const LaunchArgs&, int, int, int);
template void launch_primal_fft<float>(int, const LaunchArgs&, int);
template void launch_primal_fft<double>(int, const LaunchArgs&, int);
template void launch_fused_rows<float>(int, const LaunchArgs&, int);
template void launch_fused_rows<double>(int, const LaunchArgs&, int);
template void launch_fft<double>(int, const LaunchArgs&, int, int, int);

}  // namespace psara
