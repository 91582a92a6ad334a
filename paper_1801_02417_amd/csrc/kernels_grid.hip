// Interpolation matrix G of the measurement operator and its adjoint (Sec. 4.1, eq.
// meas_op), fused with the Stokes-to-brightness mixing L (Sec. 2.1) and the dual update
// of the data-fidelity term (Algorithm 1, l2-ball steps; radius epsilon, see the
// data-fidelity paragraph of Sec. 3.3.2).
//
// Visibilities are sorted once (at set-up) by the grid tile that holds their window start
// k0 = ceil(t - T/2).  De-gridding stages a tile plus its (T-1)-cell halo of the grid in LDS
// and lets one thread per visibility gather its T x T taps from there.  Gridding is done
// by tile owners: the workgroup of a tile walks the list of every visibility whose window
// touches the tile and accumulates the taps that fall inside it in LDS; the tile is then
// written once with plain stores, so no global atomics are used.
//
// The dual variable B is kept as B = c * Bv: the de-gridding pass writes
// Bv = B/rho2 + phi(X) - Y and the FP64 partial sums of ||Bv||^2; the gridding pass reduces
// those partials (fixed order, compensated) to c = rho2 * max(0, 1 - epsilon/||Bv||), which
// both it and the next iteration's de-gridding apply on the fly.  This equals
// B~ - rho2 P_B(Y,eps)(B~/rho2) without a second pass over the visibilities.
#include "common.hpp"
#include "launch.hpp"

namespace psara {

// ---------------------------------------------------------------------------------------------
// P6: de-grid + L mixing (+ dual B).  items: {prob, tile, first sorted vis, partial index}
template <typename R, int MODE>
__global__ void __launch_bounds__(256)
degrid_kernel(const ProbDesc* __restrict__ descs, const int4* __restrict__ items, int src_slot, int out_slot) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Cell<R>* win = (Cell<R>*)smem_raw;
  __shared__ double red[8];
  const int4 it = items[blockIdx.x];
  const ProbDesc& P = descs[it.x];
  const int K = P.K, T = P.T, ts = P.ts, nts = P.ntile_side;
  const int tile = it.y;
  const int t1 = tile / nts, t2 = tile - t1 * nts;
  const int W = ts + T - 1;
  const Cell<R>* __restrict__ grid = (const Cell<R>*)P.grid;
  const int b1 = t1 * ts, b2 = t2 * ts;
  for (int q = threadIdx.x; q < W * W; q += blockDim.x) {
    const int a = q / W, b = q - a * W;                      // a: k2 offset, b: k1 offset
    win[q] = grid[(size_t)((b2 + a) & (K - 1)) * K + ((b1 + b) & (K - 1))];
  }
  __syncthreads();

  const int vend = min(it.z + (int)blockDim.x, P.own_ptr[tile + 1]);
  const int m = it.z + threadIdx.x;
  KSum acc;
  if (m < vend) {
    const int pk = P.vis_k0[m];
    const int r1 = (pk >> 16) - b1, r2 = (pk & 0xffff) - b2;
    const V2<R> f = ((const V2<R>*)P.vis_frac)[m];
    R w1[kMaxTaps], w2[kMaxTaps];
    kb_weights<R>(f.x, T, P.deg, (const R*)P.cheb, w1);
    kb_weights<R>(f.y, T, P.deg, (const R*)P.cheb, w2);
    cplx<R> v[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = cmk(R(0), R(0));
    for (int j = 0; j < T; ++j) {
      const Cell<R>* row = win + (r2 + j) * W + r1;
      cplx<R> t[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) t[s] = cmk(R(0), R(0));
      for (int i = 0; i < T; ++i) {
        const Cell<R> c = row[i];
#pragma unroll
        for (int s = 0; s < 4; ++s) { t[s].re += w1[i] * c.s[s].re; t[s].im += w1[i] * c.s[s].im; }
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) { v[s].re += w2[j] * t[s].re; v[s].im += w2[j] * t[s].im; }
    }
    // brightness products [I+Q, U+iV, U-iV, I-Q]
    Cell<R> phi;
    phi.s[0] = cadd(v[0], v[1]);
    phi.s[1] = cadd(v[2], cmuli(v[3]));
    phi.s[2] = csub(v[2], cmuli(v[3]));
    phi.s[3] = csub(v[0], v[1]);
    Cell<R>* __restrict__ out = (Cell<R>*)P.vis[out_slot];
    if (MODE == DG_FORWARD) {
      out[m] = phi;
    } else {
      const Cell<R> y = ((const Cell<R>*)P.vis[VIS_Y])[m];
      Cell<R> o;
      if (MODE == DG_DUAL) {
        const Cell<R> bv = ((const Cell<R>*)P.vis[src_slot])[m];
        const R cb = R(P.scal[SC_CFAC] / P.rho2);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          o.s[s].re = cb * bv.s[s].re + phi.s[s].re - y.s[s].re;
          o.s[s].im = cb * bv.s[s].im + phi.s[s].im - y.s[s].im;
        }
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) o.s[s] = csub(y.s[s], phi.s[s]);
      }
      out[m] = o;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const double re = (double)o.s[s].re, im = (double)o.s[s].im;
        acc.add(re * re);
        acc.add(im * im);
      }
    }
  }
  if (MODE != DG_FORWARD) {
    const KSum tot = block_reduce(acc, red);
    if (threadIdx.x == 0) {
      P.partials[2 * it.w] = tot.s;
      P.partials[2 * it.w + 1] = tot.c;
    }
  }
}

template <typename R>
void launch_degrid(int mode, const LaunchArgs& a, int max_ts, int max_T, int src_slot, int out_slot) {
  if (a.nitems <= 0) return;
  const int W = max_ts + max_T - 1;
  const size_t shm = (size_t)W * W * sizeof(Cell<R>);
  const dim3 grid(a.nitems), block(256);
  if (mode == DG_DUAL) {
    hipLaunchKernelGGL((degrid_kernel<R, DG_DUAL>), grid, block, shm, a.stream, a.descs, a.items, src_slot, out_slot);
  } else if (mode == DG_FORWARD) {
    hipLaunchKernelGGL((degrid_kernel<R, DG_FORWARD>), grid, block, shm, a.stream, a.descs, a.items, src_slot, out_slot);
  } else {
    hipLaunchKernelGGL((degrid_kernel<R, DG_RESIDUAL>), grid, block, shm, a.stream, a.descs, a.items, src_slot, out_slot);
  }
}

// ---------------------------------------------------------------------------------------------
// P7: grid (adjoint of G, after mixing by L^H).  items: {prob, tile, writer flag, -}
// MODE GR_DUAL: scale = c from the P6 partials (stored by the writer); GR_PLAIN: scale = 1, or
// the stored c when use_cfac is set.
template <typename R, int MODE>
__global__ void __launch_bounds__(256)
grid_kernel(const ProbDesc* __restrict__ descs, const int4* __restrict__ items, int src_slot, int use_cfac) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* acc = (R*)smem_raw;                       // ts*ts cells x 8 reals
  __shared__ double red[8];
  const int4 it = items[blockIdx.x];
  const ProbDesc& P = descs[it.x];
  const int K = P.K, T = P.T, ts = P.ts, nts = P.ntile_side;
  const int tile = it.y;
  const int t1 = tile / nts, t2 = tile - t1 * nts;
  const int b1 = t1 * ts, b2 = t2 * ts;
  for (int q = threadIdx.x; q < ts * ts * 8; q += blockDim.x) acc[q] = R(0);

  R scale = R(1);
  if (MODE == GR_DUAL) {
    const double v2 = block_sum_partials(P.partials, P.n_p6, red);
    const double vn = sqrt(v2);
    const double c = (vn > P.eps) ? P.rho2 * (1.0 - P.eps / vn) : 0.0;
    scale = R(c);
    if (it.z && threadIdx.x == 0) {
      P.scal[SC_CFAC] = c;
      P.scal[SC_VNORM2] = v2;
    }
  } else if (use_cfac) {
    scale = R(P.scal[SC_CFAC]);
  }
  __syncthreads();

  const Cell<R>* __restrict__ bsrc = (const Cell<R>*)P.vis[src_slot];
  const int e0 = P.list_ptr[tile], e1 = P.list_ptr[tile + 1];
  for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int m = P.list_idx[e];
    const int pk = P.vis_k0[m];
    const int k1 = pk >> 16, k2 = pk & 0xffff;
    const V2<R> f = ((const V2<R>*)P.vis_frac)[m];
    R w1[kMaxTaps], w2[kMaxTaps];
    kb_weights<R>(f.x, T, P.deg, (const R*)P.cheb, w1);
    kb_weights<R>(f.y, T, P.deg, (const R*)P.cheb, w2);
    const Cell<R> b = bsrc[m];
    // B L^H: I = B1 + B4, Q = B1 - B4, U = B2 + B3, V = i (B3 - B2)
    cplx<R> u[4];
    u[0] = cscale(cadd(b.s[0], b.s[3]), scale);
    u[1] = cscale(csub(b.s[0], b.s[3]), scale);
    u[2] = cscale(cadd(b.s[1], b.s[2]), scale);
    u[3] = cscale(cmuli(csub(b.s[2], b.s[1])), scale);
    for (int j = 0; j < T; ++j) {
      const int c2 = (k2 + j - b2) & (K - 1);
      if (c2 >= ts) continue;
      for (int i = 0; i < T; ++i) {
        const int c1 = (k1 + i - b1) & (K - 1);
        if (c1 >= ts) continue;
        const R w = w1[i] * w2[j];
        R* cell = acc + (size_t)(c2 * ts + c1) * 8;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          atomicAdd(cell + 2 * s, w * u[s].re);
          atomicAdd(cell + 2 * s + 1, w * u[s].im);
        }
      }
    }
  }
  __syncthreads();
  Cell<R>* __restrict__ grid = (Cell<R>*)P.grid;
  for (int q = threadIdx.x; q < ts * ts; q += blockDim.x) {
    const int a = q / ts, b = q - a * ts;        // a: k2 offset, b: k1 offset
    Cell<R> c;
#pragma unroll
    for (int s = 0; s < 4; ++s) c.s[s] = cmk(acc[(size_t)q * 8 + 2 * s], acc[(size_t)q * 8 + 2 * s + 1]);
    grid[(size_t)(b2 + a) * K + (b1 + b)] = c;
  }
}

template <typename R>
void launch_grid(int mode, const LaunchArgs& a, int max_ts, int src_slot, int use_cfac) {
  if (a.nitems <= 0) return;
  const size_t shm = (size_t)max_ts * max_ts * 8 * sizeof(R);
  const dim3 grid(a.nitems), block(256);
  if (mode == GR_DUAL) {
    hipLaunchKernelGGL((grid_kernel<R, GR_DUAL>), grid, block, shm, a.stream, a.descs, a.items, src_slot, use_cfac);
  } else {
    hipLaunchKernelGGL((grid_kernel<R, GR_PLAIN>), grid, block, shm, a.stream, a.descs, a.items, src_slot, use_cfac);
  }
}

// Raise the dynamic-LDS limit of the de-grid / grid kernels once, outside any graph capture.
template <typename R>
void set_grid_kernel_limits(int max_ts, int max_T) {
  const int W = max_ts + max_T - 1;
  const int shm_dg = W * W * (int)sizeof(Cell<R>);
  const int shm_gr = max_ts * max_ts * 8 * (int)sizeof(R);
  hip_check(hipFuncSetAttribute((const void*)degrid_kernel<R, DG_DUAL>, hipFuncAttributeMaxDynamicSharedMemorySize, shm_dg), "attr");
  hip_check(hipFuncSetAttribute((const void*)degrid_kernel<R, DG_FORWARD>, hipFuncAttributeMaxDynamicSharedMemorySize, shm_dg), "attr");
  hip_check(hipFuncSetAttribute((const void*)degrid_kernel<R, DG_RESIDUAL>, hipFuncAttributeMaxDynamicSharedMemorySize, shm_dg), "attr");
  hip_check(hipFuncSetAttribute((const void*)grid_kernel<R, GR_DUAL>, hipFuncAttributeMaxDynamicSharedMemorySize, shm_gr), "attr");
  hip_check(hipFuncSetAttribute((const void*)grid_kernel<R, GR_PLAIN>, hipFuncAttributeMaxDynamicSharedMemorySize, shm_gr), "attr");
}

template void set_grid_kernel_limits<float>(int, int);
template void set_grid_kernel_limits<double>(int, int);
template void launch_degrid<float>(int, const LaunchArgs&, int, int, int, int);
template void launch_degrid<double>(int, const LaunchArgs&, int, int, int, int);
template void launch_grid<float>(int, const LaunchArgs&, int, int, int);
template void launch_grid<double>(int, const LaunchArgs&, int, int, int);

}  // namespace psara
