// Pointwise steps of Algorithm 1 (the per-pixel body is in primal.hpp) and the FP64
// reductions of the stopping quantities.
#include <algorithm>

#include "common.hpp"
#include "launch.hpp"
#include "primal.hpp"

namespace psara {

// items: {prob, block of 256 pixels, -, -}
template <typename R, int MODE>
__global__ void __launch_bounds__(256)
primal_kernel(const ProbDesc* __restrict__ descs, const int4* __restrict__ items) {
  const int4 it = items[blockIdx.x];
  const ProbDesc& P = descs[it.x];
  if (halted(P)) return;                 // stopped by an adaptive run
  const int p = it.y * 256 + threadIdx.x;
  if (p < P.n * P.n) primal_pixel<R, MODE>(P, p);
}

template <typename R>
void launch_primal(int mode, const LaunchArgs& a) {
  if (a.nitems <= 0) return;
  const dim3 g(a.nitems), b(256);
  switch (mode) {
    case PM_CONSTRAINED: hipLaunchKernelGGL((primal_kernel<R, PM_CONSTRAINED>), g, b, 0, a.stream, a.descs, a.items); break;
    case PM_INIT: hipLaunchKernelGGL((primal_kernel<R, PM_INIT>), g, b, 0, a.stream, a.descs, a.items); break;
    case PM_UNCONSTRAINED: hipLaunchKernelGGL((primal_kernel<R, PM_UNCONSTRAINED>), g, b, 0, a.stream, a.descs, a.items); break;
    case PM_TV_CONSTRAINED: hipLaunchKernelGGL((primal_kernel<R, PM_TV_CONSTRAINED>), g, b, 0, a.stream, a.descs, a.items); break;
    default: hipLaunchKernelGGL((primal_kernel<R, PM_TV_UNCONSTRAINED>), g, b, 0, a.stream, a.descs, a.items); break;
  }
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
  if (halted(P)) return;                 // stopped by an adaptive run
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
  if (halted(P)) return;                 // stopped by an adaptive run
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
  if (halted(P)) return;                 // stopped by an adaptive run
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
  if (halted(P)) return;                 // stopped by an adaptive run
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
  if (halted(P)) return;                 // stopped by an adaptive run
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
// (region < 0: the de-grid region, n_p6 pairs; count < 0: one pair per 256-pixel block of the
// problem's image, so one launch serves problems of different sizes).
__global__ void __launch_bounds__(256) finalize_kernel(const ProbDesc* __restrict__ descs, int q, int count, int scalar) {
  __shared__ double red[8];
  const ProbDesc& P = descs[blockIdx.x];
  if (halted(P)) return;                 // stopped by an adaptive run
  const double* src = (q < 0) ? P.partials : gen_part(P, q);
  const int cnt = (q < 0) ? P.n_p6 : (count < 0 ? (P.n * P.n + 255) / 256 : count);
  const double v = block_sum_partials(src, cnt, red);
  if (threadIdx.x == 0) P.scal[scalar] = v;
}

// One workgroup per problem: scal[scalar] = max of the first entries of `count` pairs of region q.
__global__ void __launch_bounds__(256) finalize_max_kernel(const ProbDesc* __restrict__ descs, int q, int count, int scalar) {
  __shared__ double red[8];
  const ProbDesc& P = descs[blockIdx.x];
  if (halted(P)) return;                 // stopped by an adaptive run
  const double* src = gen_part(P, q);
  double v = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) v = fmax(v, src[2 * i]);
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, red[w]);
    P.scal[scalar] = r;
  }
}

template <typename R>
__global__ void scale_kernel(R* p, size_t count, R factor) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    p[i] *= factor;
}

// zeta = 3 rms of the Stokes-I residual image scaled by 1/(2M)
__global__ void finalize_zeta_kernel(const ProbDesc* __restrict__ descs) {
  const ProbDesc& P = descs[blockIdx.x];
  if (halted(P)) return;                 // stopped by an adaptive run
  if (threadIdx.x == 0) {
    const double N = (double)P.n * P.n;
    P.scal[SC_ZETA] = 3.0 * sqrt(P.scal[SC_RIMG2] / N) / (2.0 * (double)P.M);
  }
}

// After a check of the stopping quantities: every problem still running adds the `chunk`
// iterations just run to scal[SC_ITERS] and is halted when the criteria of Sec. 4.6 hold:
// ||phi(S) - Y|| <= (1 + theta) epsilon, the largest relative variation of the four Stokes maps
// between the last two iterates <= the bound (a map that is zero in both counts as 0), and, if
// its bound is >= 0, N_p <= that bound (percent); a problem is also halted once its iterations
// reach scal[SC_STOP_MAXIT] when that is > 0.  active[0] = problems still running.  One
// workgroup; problems strided over its threads.
__global__ void __launch_bounds__(256) stop_decide_kernel(const ProbDesc* __restrict__ descs, int nprob, int chunk,
                                                         int* __restrict__ active) {
  __shared__ int running;
  if (threadIdx.x == 0) running = 0;
  __syncthreads();
  int mine = 0;
  for (int i = threadIdx.x; i < nprob; i += blockDim.x) {
    const ProbDesc& P = descs[i];
    if (halted(P)) continue;
    double* sc = P.scal;
    sc[SC_ITERS] += (double)chunk;
    const double res = sqrt(fmax(sc[SC_RES2], 0.0));
    double rv = 0.0;
    for (int q = 0; q < 4; ++q) {
      const double num = sqrt(fmax(sc[SC_RV0 + q], 0.0)), den = sqrt(fmax(sc[SC_SN0 + q], 0.0));
      rv = fmax(rv, den > 0.0 ? num / den : (num > 0.0 ? INFINITY : 0.0));
    }
    const double np = 100.0 * sc[SC_NPCOUNT] / ((double)P.n * P.n);
    const bool met = res <= (1.0 + sc[SC_STOP_THETA]) * P.eps && rv <= sc[SC_STOP_RV] &&
                     (sc[SC_STOP_NP] < 0.0 || np <= sc[SC_STOP_NP]);
    const bool spent = sc[SC_STOP_MAXIT] > 0.0 && sc[SC_ITERS] >= sc[SC_STOP_MAXIT];
    if (met || spent) sc[SC_HALT] = 1.0;
    else ++mine;
  }
  atomicAdd(&running, mine);
  __syncthreads();
  if (threadIdx.x == 0) active[0] = running;
}

void launch_stop_decide(const ProbDesc* descs, int nprob, int chunk, int* active, hipStream_t s) {
  hipLaunchKernelGGL(stop_decide_kernel, dim3(1), dim3(256), 0, s, descs, nprob, chunk, active);
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
void launch_finalize_max(const ProbDesc* descs, int nprob, int q, int count, int scalar, hipStream_t s) {
  hipLaunchKernelGGL(finalize_max_kernel, dim3(nprob), dim3(256), 0, s, descs, q, count, scalar);
}
template <typename R> void launch_scale(void* p, size_t count, double factor, hipStream_t s) {
  const size_t blocks = std::min<size_t>((count + 255) / 256, 4096);
  if (count > 0) hipLaunchKernelGGL((scale_kernel<R>), dim3((unsigned)blocks), dim3(256), 0, s, (R*)p, count, (R)factor);
}
void launch_finalize_zeta(const ProbDesc* descs, int nprob, hipStream_t s) {
  hipLaunchKernelGGL(finalize_zeta_kernel, dim3(nprob), dim3(64), 0, s, descs);
}

// The device-pointer data upload: *bad = 1 if any of the n doubles at y is not finite (every
// offending thread stores the same value).
__global__ void nonfinite_kernel(const double* __restrict__ y, size_t n, int* bad) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    if (!isfinite(y[i])) *bad = 1;
}
// out row p (sorted order) = y row perm[p] (the caller's order), 8 reals per row, converted to R.
template <typename R>
__global__ void gather_rows_kernel(const double* __restrict__ y, const int* __restrict__ perm, R* __restrict__ out,
                                   long long M) {
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < M * 8; q += (long long)gridDim.x * blockDim.x)
    out[q] = (R)y[(long long)perm[q >> 3] * 8 + (q & 7)];
}
template <typename R>
__global__ void to_double_kernel(const R* __restrict__ src, double* __restrict__ dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = (double)src[i];
}
void launch_nonfinite(const double* y, size_t n, int* bad, hipStream_t s) {
  const size_t blocks = std::min<size_t>((n + 255) / 256, 16384);
  if (n > 0) hipLaunchKernelGGL(nonfinite_kernel, dim3((unsigned)blocks), dim3(256), 0, s, y, n, bad);
}
template <typename R> void launch_gather_rows(const double* y, const int* perm, void* out, long long M, hipStream_t s) {
  const long long blocks = std::min<long long>((M * 8 + 255) / 256, 16384);
  if (M > 0) hipLaunchKernelGGL((gather_rows_kernel<R>), dim3((unsigned)blocks), dim3(256), 0, s, y, perm, (R*)out, M);
}
template <typename R> void launch_to_double(const void* src, double* dst, size_t n, hipStream_t s) {
  const size_t blocks = std::min<size_t>((n + 255) / 256, 16384);
  if (n > 0) hipLaunchKernelGGL((to_double_kernel<R>), dim3((unsigned)blocks), dim3(256), 0, s, (const R*)src, dst, n);
}

#define PSARA_INST(R)                                                       \
  template void launch_primal<R>(int, const LaunchArgs&);                   \
  template void launch_relvar<R>(const LaunchArgs&);                        \
  template void launch_img_sumsq<R>(const LaunchArgs&, int, int, int);      \
  template void launch_npcount<R>(const LaunchArgs&);                       \
  template void launch_img_dot<R>(const LaunchArgs&, int, int);             \
  template void launch_img_scale<R>(const LaunchArgs&, int, int, int);      \
  template void launch_fill<R>(void*, size_t, hipStream_t);                 \
  template void launch_scale<R>(void*, size_t, double, hipStream_t);       \
  template void launch_gather_rows<R>(const double*, const int*, void*, long long, hipStream_t); \
  template void launch_to_double<R>(const void*, double*, size_t, hipStream_t);
PSARA_INST(float)
PSARA_INST(double)
#undef PSARA_INST

}  // namespace psara
