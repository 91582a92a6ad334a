// Per-pixel primal step of Algorithm 1, shared by the stand-alone primal kernel and the
// fused primal + row-FFT kernel.
//
// For pixel p: the primal update of S (projection on U, or U' for the initialisation and
// the unconstrained problem; eq. real_proj, eq. pos_set) and Z (projection on V, eq. set_V),
// the over-relaxed point X = 2 S_new - S, the epigraphical dual updates of C and D
// (projections on E1 = epi h1 and E2 = epi h2, eqs. proj_e1, proj_e2_def, with the boundary
// readings "<=" and r = 0, d = 0 -> 0), and the Dirac block of the sparsity dual
// (A_dirac = clip(A_dirac + rho1 X / sqrt(nb), -gW, gW)).  The C/D updates depend only on X
// and Z, so running them here rather than after the A and B updates gives the same iterate.
#pragma once

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

// What the primal step of pixel p reads besides the data term's gradient, requested by
// primal_load (so a caller can issue the loads early and use them later).
template <typename R>
struct PrimalIn {
  V4<R> s, pa, pb, ad, gw, c;
  V2<R> z, d;
};

template <typename R, int MODE>
__device__ inline PrimalIn<R> primal_load(const ProbDesc& P, int p) {
  PrimalIn<R> in{};
  in.s = ((const V4<R>*)P.img[IMG_S])[p];
  if (MODE != PM_INIT) {
    in.pa = ((const V4<R>*)P.img[IMG_PSIA])[p];
    if (!pm_tv(MODE)) in.pb = ((const V4<R>*)P.img[IMG_PSIA2])[p];
    if (P.has_dirac) {
      in.ad = ((const V4<R>*)P.coef[COEF_A])[p];
      in.gw = ((const V4<R>*)P.coef[COEF_GW])[p];
    }
  }
  if (pm_constrained(MODE)) {
    in.c = ((const V4<R>*)P.img[IMG_C])[p];
    in.z = ((const V2<R>*)P.img[IMG_Z])[p];
    in.d = ((const V2<R>*)P.img[IMG_D])[p];
  }
  return in;
}

// Updates every per-pixel variable of pixel p in place from its inputs `in` and returns X
// (S_new in the TV modes); g is Re phi^dagger B at p (the data term's gradient in the TV modes).
template <typename R, int MODE>
__device__ inline V4<R> primal_pixel_in(const ProbDesc& P, int p, V4<R> g, const PrimalIn<R>& in) {
  const R tau = R(P.tau), nm = R(P.norm);
  V4<R>* S = (V4<R>*)P.img[IMG_S];
  V4<R>* X = (V4<R>*)P.img[IMG_X];
  const V4<R> s = in.s;
  V4<R> ad;
  const bool dirac = (MODE != PM_INIT) && P.has_dirac;
  if (MODE != PM_INIT) {
    const V4<R> pa = in.pa;
    g.x += pa.x; g.y += pa.y; g.z += pa.z; g.w += pa.w;
    if (!pm_tv(MODE)) {
      const V4<R> pb = in.pb;
      g.x += pb.x; g.y += pb.y; g.z += pb.z; g.w += pb.w;
    }
    if (dirac) {
      ad = in.ad;
      g.x += nm * ad.x; g.y += nm * ad.y; g.z += nm * ad.z; g.w += nm * ad.w;
    }
  }
  V4<R> c;
  if (pm_constrained(MODE)) {
    c = in.c;
    g.x += c.x; g.y += c.y; g.z += c.z; g.w += c.w;
  }
  V4<R> sn;
  sn.x = s.x - tau * g.x; sn.y = s.y - tau * g.y; sn.z = s.z - tau * g.z; sn.w = s.w - tau * g.w;
  if (pm_positive_I(MODE)) sn.x = fmax(sn.x, R(0));          // U': Stokes I >= 0
  V4<R> x;
  x.x = R(2) * sn.x - s.x; x.y = R(2) * sn.y - s.y; x.z = R(2) * sn.z - s.z; x.w = R(2) * sn.w - s.w;
  S[p] = sn;
  X[p] = x;
  if (dirac) {
    const V4<R> gw = in.gw;
    const R r1 = R(P.rho1) * nm;
    ad.x = fmin(fmax(ad.x + r1 * x.x, -gw.x), gw.x);
    ad.y = fmin(fmax(ad.y + r1 * x.y, -gw.y), gw.y);
    ad.z = fmin(fmax(ad.z + r1 * x.z, -gw.z), gw.z);
    ad.w = fmin(fmax(ad.w + r1 * x.w, -gw.w), gw.w);
    ((V4<R>*)P.coef[COEF_A])[p] = ad;
  }
  if (pm_constrained(MODE)) {
    V2<R>* Z = (V2<R>*)P.img[IMG_Z];
    V2<R>* D = (V2<R>*)P.img[IMG_D];
    const V2<R> z = in.z, d = in.d;
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
  return pm_tv(MODE) ? sn : x;    // Algorithm 3 transforms S_new for its next gradient
}

template <typename R, int MODE>
__device__ inline V4<R> primal_pixel_g(const ProbDesc& P, int p, V4<R> g) {
  return primal_pixel_in<R, MODE>(P, p, g, primal_load<R, MODE>(P, p));
}

// The same with Re phi^dagger B read from its image.
template <typename R, int MODE>
__device__ inline V4<R> primal_pixel(const ProbDesc& P, int p) {
  return primal_pixel_g<R, MODE>(P, p, ((const V4<R>*)P.img[IMG_PHIB])[p]);
}

}  // namespace psara
