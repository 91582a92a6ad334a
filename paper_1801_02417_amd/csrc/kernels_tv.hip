// TV and l1 + TV priors of Algorithm 3 (Sec. 4.3): Psi^dagger = [d1; d2] or [1; d1; d2] with
// d1, d2 the forward differences along the two image axes (zero at the last row / column),
// and the dual step A = A~ - rho1 T(A~ / rho1) with T the proximity operator of the weighted
// norm: on each pixel's gradient pair the l2,1 norm's (group soft thresholding), which makes
// the step the projection of the pair A~ = A + rho1 Psi^dagger X on the disc of radius mu_i,
// and on the Dirac block the soft threshold, i.e. clip(A~, -upsilon_i, upsilon_i).
// The dual A is stored as N x 4 blocks: [d1, d2] (TV) or [Dirac, d1, d2] (l1 + TV).
#include "common.hpp"
#include "launch.hpp"

namespace psara {

// the dual step at every pixel of the item's block (reads X at the pixel and its two forward
// neighbours, writes only the pixel's own dual entries, so workgroups do not interact)
template <typename R>
__global__ void __launch_bounds__(256) tv_dual_kernel(const ProbDesc* __restrict__ descs, const int4* __restrict__ items) {
  const int4 it = items[blockIdx.x];
  const ProbDesc& P = descs[it.x];
  if (halted(P)) return;                 // stopped by an adaptive run
  const int n = P.n, N = n * n, p = it.y * 256 + threadIdx.x;
  if (p >= N) return;
  const int r = p / n, c = p - r * n;
  const V4<R>* __restrict__ X = (const V4<R>*)P.img[IMG_X];
  V4<R>* __restrict__ A = (V4<R>*)P.coef[COEF_A];
  const R r1 = R(P.rho1);
  const V4<R> x = X[p];
  const V4<R> xd = r < n - 1 ? X[p + n] : x;          // zero difference on the last row
  const V4<R> xr = c < n - 1 ? X[p + 1] : x;          // and on the last column
  const R g1[4] = {xd.x - x.x, xd.y - x.y, xd.z - x.z, xd.w - x.w};
  const R g2[4] = {xr.x - x.x, xr.y - x.y, xr.z - x.z, xr.w - x.w};
  const int o = P.tv_kind == 2 ? N : 0;               // the d1 block follows the Dirac block
  const V4<R> a1 = A[o + p], a2 = A[o + N + p];
  R t1[4] = {a1.x, a1.y, a1.z, a1.w}, t2[4] = {a2.x, a2.y, a2.z, a2.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    t1[i] += r1 * g1[i];
    t2[i] += r1 * g2[i];
    const R mu = R(P.tvw[i]);
    const R nrm = sqrt(t1[i] * t1[i] + t2[i] * t2[i]);
    if (nrm > mu) {
      const R f = mu / nrm;
      t1[i] *= f;
      t2[i] *= f;
    }
  }
  A[o + p] = V4<R>{t1[0], t1[1], t1[2], t1[3]};
  A[o + N + p] = V4<R>{t2[0], t2[1], t2[2], t2[3]};
  if (P.tv_kind == 2) {
    const V4<R> a0 = A[p];
    const R xs[4] = {x.x, x.y, x.z, x.w};
    R t0[4] = {a0.x, a0.y, a0.z, a0.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const R u = R(P.l1w[i]);
      t0[i] = fmin(fmax(t0[i] + r1 * xs[i], -u), u);
    }
    A[p] = V4<R>{t0[0], t0[1], t0[2], t0[3]};
  }
}

// Psi A = [A0] + d1^T A1 + d2^T A2 into IMG_PSIA, with (d^T g)(j) = g(j - 1) - g(j) where
// each term exists (the first index has no predecessor, the last carries no difference)
template <typename R>
__global__ void __launch_bounds__(256) tv_synth_kernel(const ProbDesc* __restrict__ descs, const int4* __restrict__ items) {
  const int4 it = items[blockIdx.x];
  const ProbDesc& P = descs[it.x];
  if (halted(P)) return;                 // stopped by an adaptive run
  const int n = P.n, N = n * n, p = it.y * 256 + threadIdx.x;
  if (p >= N) return;
  const int r = p / n, c = p - r * n;
  const V4<R>* __restrict__ A = (const V4<R>*)P.coef[COEF_A];
  const int b1 = P.tv_kind == 2 ? N : 0, b2 = b1 + N;    // the d1 and d2 blocks
  V4<R> o = P.tv_kind == 2 ? A[p] : V4<R>{R(0), R(0), R(0), R(0)};
  auto add = [&](const V4<R>& v, R s) { o.x += s * v.x; o.y += s * v.y; o.z += s * v.z; o.w += s * v.w; };
  if (r >= 1) add(A[b1 + p - n], R(1));
  if (r < n - 1) add(A[b1 + p], R(-1));
  if (c >= 1) add(A[b2 + p - 1], R(1));
  if (c < n - 1) add(A[b2 + p], R(-1));
  ((V4<R>*)P.img[IMG_PSIA])[p] = o;
}

// partial sums of sum_i mu_i ||grad S_i(p)|| (+ upsilon_i |S_i(p)|) over the block (region 0)
template <typename R>
__global__ void __launch_bounds__(256) tv_objective_kernel(const ProbDesc* __restrict__ descs, const int4* __restrict__ items) {
  __shared__ double red[8];
  const int4 it = items[blockIdx.x];
  const ProbDesc& P = descs[it.x];
  if (halted(P)) return;                 // stopped by an adaptive run
  const int n = P.n, N = n * n, p = it.y * 256 + threadIdx.x;
  KSum k;
  if (p < N) {
    const int r = p / n, c = p - r * n;
    const V4<R>* __restrict__ S = (const V4<R>*)P.img[IMG_S];
    const V4<R> s = S[p];
    const V4<R> sd = r < n - 1 ? S[p + n] : s;
    const V4<R> sr = c < n - 1 ? S[p + 1] : s;
    const double v[4] = {s.x, s.y, s.z, s.w};
    const double d[4] = {(double)sd.x - s.x, (double)sd.y - s.y, (double)sd.z - s.z, (double)sd.w - s.w};
    const double e[4] = {(double)sr.x - s.x, (double)sr.y - s.y, (double)sr.z - s.z, (double)sr.w - s.w};
    for (int i = 0; i < 4; ++i) {
      k.add(P.tvw[i] * sqrt(d[i] * d[i] + e[i] * e[i]));
      if (P.tv_kind == 2) k.add(P.l1w[i] * fabs(v[i]));
    }
  }
  const KSum t = block_reduce(k, red);
  if (threadIdx.x == 0) {
    double* g = P.partials + 2 * (size_t)P.n_p6;
    g[2 * it.y] = t.s;
    g[2 * it.y + 1] = t.c;
  }
}

template <typename R> void launch_tv_dual(const LaunchArgs& a) {
  if (a.nitems > 0) hipLaunchKernelGGL((tv_dual_kernel<R>), dim3(a.nitems), dim3(256), 0, a.stream, a.descs, a.items);
}
template <typename R> void launch_tv_synth(const LaunchArgs& a) {
  if (a.nitems > 0) hipLaunchKernelGGL((tv_synth_kernel<R>), dim3(a.nitems), dim3(256), 0, a.stream, a.descs, a.items);
}
template <typename R> void launch_tv_objective(const LaunchArgs& a) {
  if (a.nitems > 0) hipLaunchKernelGGL((tv_objective_kernel<R>), dim3(a.nitems), dim3(256), 0, a.stream, a.descs, a.items);
}

template void launch_tv_dual<float>(const LaunchArgs&);
template void launch_tv_dual<double>(const LaunchArgs&);
template void launch_tv_synth<float>(const LaunchArgs&);
template void launch_tv_synth<double>(const LaunchArgs&);
template void launch_tv_objective<float>(const LaunchArgs&);
template void launch_tv_objective<double>(const LaunchArgs&);

}  // namespace psara
