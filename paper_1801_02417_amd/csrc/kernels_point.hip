// Pointwise steps of Algorithm 1 and the FP64 reductions of the stopping quantities.
//
// P1 fuses, per pixel, the primal updates of S (projection on U, or U' for the
// initialisation and the unconstrained problem; eq. real_proj, eq. pos_set) and Z
// (projection on V, eq. set_V), the over-relaxed point X = 2 S_new - S, the epigraphical
// dual updates of C and D (projections on E1 = epi h1 and E2 = epi h2, eqs. proj_e1,
// proj_e2_def, with the boundary readings "<=" and r = 0, d = 0 -> 0), and the Dirac block
// of the sparsity dual (A_dirac = clip(A_dirac + rho1 X / sqrt(nb), -gW, gW)).  The C/D
// updates depend only on X and Z, so running them here rather than after the A and B
// updates gives the same iterate.
#include "common.hpp"
#include "launch.hpp"

namespace psara {

template <typename R>
__device__ inline void proj_E1(R c, R d, R& pc, R& pd) {
  if (c + d >= R(0)) { pc = c; pd = d; }
  else { pc = R(0.5) * (c - d); pd = R(0.5) * (d - c); }
}

template <typename R>
__device__ inline void proj_E2(R r0, R r1, R r2, R d, R& p0, R& p1, R& p2, R& pd) {
  const R nr = sqrt(r0 * r0 + r1 * r1 + r2 * r2);
  if (nr <= d) { p0 = r0; p1 = r1; p2 = r2; pd = d; }
  else if (nr <= -d) { p0 = p1 = p2 = pd = R(0); }
  else {
    const R a = R(0.5) * (R(1) + d / nr);
    p0 = a * r0; p1 = a * r1; p2 = a * r2; pd = a * nr;
  }
}

// items: {prob, block of 256 pixels, -, -}
template <typename R, int MODE>
__global__ void __launch_bounds__(256)
primal_kernel(const ProbDesc* __restrict__ descs, const int4* __restrict__ items) {
  const int4 it = items[blockIdx.x];
  const ProbDesc& P = descs[it.x];
  const int N = P.n * P.n;
  const int p = it.y * 256 + threadIdx.x;
  if (p >= N) return;
  const R tau = R(P.tau), nm = R(P.norm);
  V4<R>* S = (V4<R>*)P.img[IMG_S];
  V4<R>* X = (V4<R>*)P.img[IMG_X];
  const V4<R> s = S[p];
  V4<R> g = ((const V4<R>*)P.img[IMG_PHIB])[p];
  V4<R> ad;
  const bool dirac = (MODE != PM_INIT) && P.has_dirac;
  if (MODE != PM_INIT) {
    const V4<R> pa = ((const V4<R>*)P.img[IMG_PSIA])[p];
    g.x += pa.x; g.y += pa.y; g.z += pa.z; g.w += pa.w;
    if (dirac) {
      ad = ((const V4<R>*)P.coef[COEF_A])[p];
      g.x += nm * ad.x; g.y += nm * ad.y; g.z += nm * ad.z; g.w += nm * ad.w;
    }
  }
  V4<R> c;
  if (MODE == PM_CONSTRAINED) {
    c = ((const V4<R>*)P.img[IMG_C])[p];
    g.x += c.x; g.y += c.y; g.z += c.z; g.w += c.w;
  }
  V4<R> sn;
  sn.x = s.x - tau * g.x; sn.y = s.y - tau * g.y; sn.z = s.z - tau * g.z; sn.w = s.w - tau * g.w;
  if (MODE != PM_CONSTRAINED) sn.x = fmax(sn.x, R(0));       // U': Stokes I >= 0
  V4<R> x;
  x.x = R(2) * sn.x - s.x; x.y = R(2) * sn.y - s.y; x.z = R(2) * sn.z - s.z; x.w = R(2) * sn.w - s.w;
  S[p] = sn;
  X[p] = x;
  if (dirac) {
    const V4<R> gw = ((const V4<R>*)P.coef[COEF_GW])[p];
    const R r1 = R(P.rho1) * nm;
    ad.x = fmin(fmax(ad.x + r1 * x.x, -gw.x), gw.x);
    ad.y = fmin(fmax(ad.y + r1 * x.y, -gw.y), gw.y);
    ad.z = fmin(fmax(ad.z + r1 * x.z, -gw.z), gw.z);
    ad.w = fmin(fmax(ad.w + r1 * x.w, -gw.w), gw.w);
    ((V4<R>*)P.coef[COEF_A])[p] = ad;
  }
  if (MODE == PM_CONSTRAINED) {
    V2<R>* Z = (V2<R>*)P.img[IMG_Z];
    V2<R>* D = (V2<R>*)P.img[IMG_D];
    const V2<R> z = Z[p], d = D[p];
    // Z = P_V(Z - tau D)
    V2<R> zt, zn;
    zt.x = z.x - tau * d.x; zt.y = z.y - tau * d.y;
    if (zt.x + zt.y <= R(0)) zn = zt;
    else { zn.x = R(0.5) * (zt.x - zt.y); zn.y = R(0.5) * (zt.y - zt.x); }
    const R r3 = R(P.rho3), ir3 = R(1) / r3;
    V4<R> ct;
    ct.x = c.x + r3 * x.x; ct.y = c.y + r3 * x.y; ct.z = c.z + r3 * x.z; ct.w = c.w + r3 * x.w;
    V2<R> dt;
    dt.x = d.x + r3 * (R(2) * zn.x - z.x);
    dt.y = d.y + r3 * (R(2) * zn.y - z.y);
    R pc, pd;
    proj_E1<R>(ct.x * ir3, dt.x * ir3, pc, pd);
    V4<R> cn;
    V2<R> dn;
    cn.x = ct.x - r3 * pc;
    dn.x = dt.x - r3 * pd;
    R p0, p1, p2, pd2;
    proj_E2<R>(ct.y * ir3, ct.z * ir3, ct.w * ir3, dt.y * ir3, p0, p1, p2, pd2);
    cn.y = ct.y - r3 * p0; cn.z = ct.z - r3 * p1; cn.w = ct.w - r3 * p2;
    dn.y = dt.y - r3 * pd2;
    ((V4<R>*)P.img[IMG_C])[p] = cn;
    Z[p] = zn;
    D[p] = dn;
  }
}

template <typename R>
void launch_primal(int mode, const LaunchArgs& a) {
  if (a.nitems <= 0) return;
  const dim3 g(a.nitems), b(256);
  if (mode == PM_CONSTRAINED) hipLaunchKernelGGL((primal_kernel<R, PM_CONSTRAINED>), g, b, 0, a.stream, a.descs, a.items);
  else if (mode == PM_INIT) hipLaunchKernelGGL((primal_kernel<R, PM_INIT>), g, b, 0, a.stream, a.descs, a.items);
  else hipLaunchKernelGGL((primal_kernel<R, PM_UNCONSTRAINED>), g, b, 0, a.stream, a.descs, a.items);
}

// ---------------------------------------------------------------------------------------------
// Reductions.  Every workgroup writes (sum, compensation) pairs into the generic partial
// regions q * gen_stride + it.y; `launch_finalize` sums them in a fixed order.
__device__ inline double* gen_part(const ProbDesc& P, int q) {
  return P.partials + 2 * (size_t)P.n_p6 + 2 * (size_t)q * P.gen_stride;
}

// relative variation: ||X - S||^2 (q = 0..3) and ||2S - X||^2 (q = 4..7) per Stokes map; with
// X = 2 S_new - S_old and S = S_new these are ||S_new - S_old||^2 and ||S_old||^2.
template <typename R>
__global__ void __launch_bounds__(256) relvar_kernel(const ProbDesc* __restrict__ descs, const int4* __restrict__ items) {
  __shared__ double red[8];
  const int4 it = items[blockIdx.x];
  const ProbDesc& P = descs[it.x];
  const int N = P.n * P.n, p = it.y * 256 + threadIdx.x;
  KSum k[8];
  if (p < N) {
    const V4<R> s = ((const V4<R>*)P.img[IMG_S])[p];
    const V4<R> x = ((const V4<R>*)P.img[IMG_X])[p];
    const double d[4] = {(double)x.x - s.x, (double)x.y - s.y, (double)x.z - s.z, (double)x.w - s.w};
    const double o[4] = {2.0 * s.x - x.x, 2.0 * s.y - x.y, 2.0 * s.z - x.z, 2.0 * s.w - x.w};
    for (int i = 0; i < 4; ++i) { k[i].add(d[i] * d[i]); k[4 + i].add(o[i] * o[i]); }
  }
  for (int q = 0; q < 8; ++q) {
    const KSum t = block_reduce(k[q], red);
    if (threadIdx.x == 0) { double* g = gen_part(P, q); g[2 * it.y] = t.s; g[2 * it.y + 1] = t.c; }
  }
}

// sum of squares of one channel of an image slot (q = 0)
template <typename R>
__global__ void __launch_bounds__(256) img_sumsq_kernel(const ProbDesc* __restrict__ descs, const int4* __restrict__ items, int slot, int ch) {
  __shared__ double red[8];
  const int4 it = items[blockIdx.x];
  const ProbDesc& P = descs[it.x];
  const int N = P.n * P.n, p = it.y * 256 + threadIdx.x;
  KSum k;
  if (p < N) {
    const R* v = (const R*)P.img[slot] + 4 * (size_t)p;
    const double a = (double)v[ch];
    k.add(a * a);
  }
  const KSum t = block_reduce(k, red);
  if (threadIdx.x == 0) { double* g = gen_part(P, 0); g[2 * it.y] = t.s; g[2 * it.y + 1] = t.c; }
}

// count of pixels with ||S_{n,2:4}|| - S_{n,1} > zeta (q = 0)
template <typename R>
__global__ void __launch_bounds__(256) npcount_kernel(const ProbDesc* __restrict__ descs, const int4* __restrict__ items) {
  __shared__ double red[8];
  const int4 it = items[blockIdx.x];
  const ProbDesc& P = descs[it.x];
  const int N = P.n * P.n, p = it.y * 256 + threadIdx.x;
  KSum k;
  if (p < N) {
    const V4<R> s = ((const V4<R>*)P.img[IMG_S])[p];
    const double v = sqrt((double)s.y * s.y + (double)s.z * s.z + (double)s.w * s.w) - (double)s.x;
    if (v > P.scal[SC_ZETA]) k.add(1.0);
  }
  const KSum t = block_reduce(k, red);
  if (threadIdx.x == 0) { double* g = gen_part(P, 0); g[2 * it.y] = t.s; g[2 * it.y + 1] = t.c; }
}

// <x, y> (q = 0) and ||y||^2 (q = 1) over all four channels
template <typename R>
__global__ void __launch_bounds__(256) img_dot_kernel(const ProbDesc* __restrict__ descs, const int4* __restrict__ items, int xs, int ys) {
  __shared__ double red[8];
  const int4 it = items[blockIdx.x];
  const ProbDesc& P = descs[it.x];
  const int N = P.n * P.n, p = it.y * 256 + threadIdx.x;
  KSum kd, kn;
  if (p < N) {
    const V4<R> x = ((const V4<R>*)P.img[xs])[p];
    const V4<R> y = ((const V4<R>*)P.img[ys])[p];
    kd.add((double)x.x * y.x); kd.add((double)x.y * y.y); kd.add((double)x.z * y.z); kd.add((double)x.w * y.w);
    kn.add((double)y.x * y.x); kn.add((double)y.y * y.y); kn.add((double)y.z * y.z); kn.add((double)y.w * y.w);
  }
  KSum t = block_reduce(kd, red);
  if (threadIdx.x == 0) { double* g = gen_part(P, 0); g[2 * it.y] = t.s; g[2 * it.y + 1] = t.c; }
  t = block_reduce(kn, red);
  if (threadIdx.x == 0) { double* g = gen_part(P, 1); g[2 * it.y] = t.s; g[2 * it.y + 1] = t.c; }
}

// dst = src / sqrt(scal[scalar])
template <typename R>
__global__ void __launch_bounds__(256) img_scale_kernel(const ProbDesc* __restrict__ descs, const int4* __restrict__ items, int dst, int src, int scalar) {
  const int4 it = items[blockIdx.x];
  const ProbDesc& P = descs[it.x];
  const int N = P.n * P.n, p = it.y * 256 + threadIdx.x;
  if (p >= N) return;
  const double nv = P.scal[scalar];
  const R f = R(nv > 0.0 ? 1.0 / sqrt(nv) : 0.0);
  V4<R> v = ((const V4<R>*)P.img[src])[p];
  v.x *= f; v.y *= f; v.z *= f; v.w *= f;
  ((V4<R>*)P.img[dst])[p] = v;
}

template <typename R>
__global__ void fill_kernel(R* p, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) p[i] = R(0);
}

// One workgroup per problem: scal[scalar] = sum of `count` pairs of generic region q
// (region < 0: the de-grid region, n_p6 pairs).
__global__ void __launch_bounds__(256) finalize_kernel(const ProbDesc* __restrict__ descs, int q, int count, int scalar) {
  __shared__ double red[8];
  const ProbDesc& P = descs[blockIdx.x];
  const double* src = (q < 0) ? P.partials : gen_part(P, q);
  const int cnt = (q < 0) ? P.n_p6 : count;
  const double v = block_sum_partials(src, cnt, red);
  if (threadIdx.x == 0) P.scal[scalar] = v;
}

// zeta = 3 rms of the Stokes-I residual image scaled by 1/(2M)
__global__ void finalize_zeta_kernel(const ProbDesc* __restrict__ descs) {
  const ProbDesc& P = descs[blockIdx.x];
  if (threadIdx.x == 0) {
    const double N = (double)P.n * P.n;
    P.scal[SC_ZETA] = 3.0 * sqrt(P.scal[SC_RIMG2] / N) / (2.0 * (double)P.M);
  }
}

template <typename R> void launch_relvar(const LaunchArgs& a) {
  if (a.nitems > 0) hipLaunchKernelGGL((relvar_kernel<R>), dim3(a.nitems), dim3(256), 0, a.stream, a.descs, a.items);
}
template <typename R> void launch_img_sumsq(const LaunchArgs& a, int slot, int channel, int) {
  if (a.nitems > 0) hipLaunchKernelGGL((img_sumsq_kernel<R>), dim3(a.nitems), dim3(256), 0, a.stream, a.descs, a.items, slot, channel);
}
template <typename R> void launch_npcount(const LaunchArgs& a) {
  if (a.nitems > 0) hipLaunchKernelGGL((npcount_kernel<R>), dim3(a.nitems), dim3(256), 0, a.stream, a.descs, a.items);
}
template <typename R> void launch_img_dot(const LaunchArgs& a, int xs, int ys) {
  if (a.nitems > 0) hipLaunchKernelGGL((img_dot_kernel<R>), dim3(a.nitems), dim3(256), 0, a.stream, a.descs, a.items, xs, ys);
}
template <typename R> void launch_img_scale(const LaunchArgs& a, int dst, int src, int scalar) {
  if (a.nitems > 0) hipLaunchKernelGGL((img_scale_kernel<R>), dim3(a.nitems), dim3(256), 0, a.stream, a.descs, a.items, dst, src, scalar);
}
template <typename R> void launch_fill(void* p, size_t count, hipStream_t s) {
  if (count == 0) return;
  const size_t blocks = std::min<size_t>((count + 255) / 256, 65536);
  hipLaunchKernelGGL((fill_kernel<R>), dim3((unsigned)blocks), dim3(256), 0, s, (R*)p, count);
}
void launch_finalize(const ProbDesc* descs, int nprob, int q, int count, int scalar, hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3(nprob), dim3(256), 0, s, descs, q, count, scalar);
}
void launch_finalize_zeta(const ProbDesc* descs, int nprob, hipStream_t s) {
  hipLaunchKernelGGL(finalize_zeta_kernel, dim3(nprob), dim3(64), 0, s, descs);
}

#define PSARA_INST(R)                                                       \
  template void launch_primal<R>(int, const LaunchArgs&);                   \
  template void launch_relvar<R>(const LaunchArgs&);                        \
  template void launch_img_sumsq<R>(const LaunchArgs&, int, int, int);      \
  template void launch_npcount<R>(const LaunchArgs&);                       \
  template void launch_img_dot<R>(const LaunchArgs&, int, int);             \
  template void launch_img_scale<R>(const LaunchArgs&, int, int, int);      \
  template void launch_fill<R>(void*, size_t, hipStream_t);
PSARA_INST(float)
PSARA_INST(double)
#undef PSARA_INST

}  // namespace psara
