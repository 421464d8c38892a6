// geom.h -- device arithmetic of the diamond lattice (FP64, no contraction).
//
// Paper (Blanco-Pillado, Olum, Shlaer), Section "Semi-parallel cosmic string
// simulation": the world sheet of x(sigma,t) = [a(t-sigma) + b(t+sigma)]/2 with
// piecewise-linear a, b is a union of diamonds; in flat space each diamond is planar
// (and the evolution exact), in an expanding universe expansion is applied at first
// order in each diamond. Intersections between pieces of string are found and the
// strings exchange partners.
//
// Every expression below is evaluated exactly as parenthesised: the translation
// unit is compiled with -ffp-contract=off and `#pragma clang fp contract(off)`.
#pragma once
#include <hip/hip_runtime.h>

#pragma clang fp contract(off)

namespace sp {

struct V4 {
  double x, y, z, t;
};

// Diamond with bottom B = X[n-1][j], left L = X[n][k], right R = X[n][j]
// (j = next[k]); returns the top X[n+1][k].
// Flat space: the diamond is a parallelogram, T = L + (R - B) per component.
__device__ __forceinline__ V4 top_flat(const V4& L, const V4& R, const V4& B) {
  V4 T;
  T.x = L.x + (R.x - B.x);
  T.y = L.y + (R.y - B.y);
  T.z = L.z + (R.z - B.z);
  T.t = L.t + (R.t - B.t);
  return T;
}

// Periodic box of side `box`. nearest(d) = rint(d / box), the number of periods in d
// rounded half to even. When box is a power of two, 1/box is exact and d * (1/box)
// equals d / box bit for bit, so the division is replaced by a multiplication.
struct Period {
  double box, inv;
  int pow2;
  __device__ __forceinline__ double nearest(double d) const {
    return pow2 ? rint(d * inv) : rint(d / box);
  }
};

__device__ __forceinline__ double min_image(double d, const Period& P) {
  return d - P.box * P.nearest(d);
}

// Expanding universe (conformal time), first order per diamond, H = hcoef / eta_m with
// eta_m the mean time of L and R. dL = L - B (minimum image), dR = R - B (same point),
// alpha = t_L - t_B, beta = t_R - t_B:
//   x_T = (x_L + dR) - H (beta dL + alpha dR)
//   t_T = (t_L + beta) - H (alpha beta + dL.dR)
// Both future edges transported across the diamond under
//   dp/deta = -H [q - (p.q) p],  dq/deta = -H [p - (p.q) q]
// (p, q the unit null directions of the world sheet) meet at this top.
__device__ __forceinline__ V4 top_frw(const V4& L, const V4& R, const V4& B, const Period& P,
                                      double hcoef) {
  const double dLx = min_image(L.x - B.x, P);
  const double dLy = min_image(L.y - B.y, P);
  const double dLz = min_image(L.z - B.z, P);
  const double dRx = R.x - B.x;
  const double dRy = R.y - B.y;
  const double dRz = R.z - B.z;
  const double alpha = L.t - B.t;
  const double beta = R.t - B.t;
  const double eta_m = 0.5 * (L.t + R.t);
  const double H = hcoef / eta_m;
  V4 T;
  T.x = (L.x + dRx) - H * (beta * dLx + alpha * dRx);
  T.y = (L.y + dRy) - H * (beta * dLy + alpha * dRy);
  T.z = (L.z + dRz) - H * (beta * dLz + alpha * dRz);
  const double dLdR = (dLx * dRx + dLy * dRy) + dLz * dRz;
  T.t = (L.t + beta) - H * ((alpha * beta) + dLdR);
  return T;
}

template <bool FRW>
__device__ __forceinline__ V4 top(const V4& L, const V4& R, const V4& B, const Period& P,
                                  double hcoef) {
  if constexpr (FRW)
    return top_frw(L, R, B, P, hcoef);
  else
    return top_flat(L, R, B);
}

// ---- element of band n: strip between k and j = next[k] from slice n to n+1 -------
// Vertices v0 = X[n][k], v1 = X[n][j] - s, v2 = X[n+1][k], v3 = X[n+1][j] - s with
// s = box * rint((X[n][j] - X[n][k]) / box) (spatial), triangles U = (v0, v1, v2) and
// D = (v2, v1, v3).
struct Elem {
  V4 v[4];
};

__device__ __forceinline__ Elem make_elem(const V4& Lk, const V4& Lj, const V4& Tk, const V4& Tj,
                                          const Period& P) {
  const double sx = P.box * P.nearest(Lj.x - Lk.x);
  const double sy = P.box * P.nearest(Lj.y - Lk.y);
  const double sz = P.box * P.nearest(Lj.z - Lk.z);
  Elem e;
  e.v[0] = Lk;
  e.v[1] = V4{Lj.x - sx, Lj.y - sy, Lj.z - sz, Lj.t};
  e.v[2] = Tk;
  e.v[3] = V4{Tj.x - sx, Tj.y - sy, Tj.z - sz, Tj.t};
  return e;
}

struct Box4 {
  double lo[4], hi[4];
};

__device__ __forceinline__ Box4 elem_box(const Elem& e) {
  Box4 b;
  b.lo[0] = fmin(fmin(e.v[0].x, e.v[1].x), fmin(e.v[2].x, e.v[3].x));
  b.lo[1] = fmin(fmin(e.v[0].y, e.v[1].y), fmin(e.v[2].y, e.v[3].y));
  b.lo[2] = fmin(fmin(e.v[0].z, e.v[1].z), fmin(e.v[2].z, e.v[3].z));
  b.lo[3] = fmin(fmin(e.v[0].t, e.v[1].t), fmin(e.v[2].t, e.v[3].t));
  b.hi[0] = fmax(fmax(e.v[0].x, e.v[1].x), fmax(e.v[2].x, e.v[3].x));
  b.hi[1] = fmax(fmax(e.v[0].y, e.v[1].y), fmax(e.v[2].y, e.v[3].y));
  b.hi[2] = fmax(fmax(e.v[0].z, e.v[1].z), fmax(e.v[2].z, e.v[3].z));
  b.hi[3] = fmax(fmax(e.v[0].t, e.v[1].t), fmax(e.v[2].t, e.v[3].t));
  return b;
}

// ---- 4x4 determinants through the 2x2 minors of rows (x,y) and (z,t) --------------
__device__ __forceinline__ double mxy(const V4& u, const V4& v) { return u.x * v.y - u.y * v.x; }
__device__ __forceinline__ double mzt(const V4& u, const V4& v) { return u.z * v.t - u.t * v.z; }

__device__ __forceinline__ double det4(const V4& a, const V4& b, const V4& c, const V4& d) {
  double r = mxy(a, b) * mzt(c, d);
  r = r - mxy(a, c) * mzt(b, d);
  r = r + mxy(a, d) * mzt(b, c);
  r = r + mxy(b, c) * mzt(a, d);
  r = r - mxy(b, d) * mzt(a, c);
  r = r + mxy(c, d) * mzt(a, b);
  return r;
}

__device__ __forceinline__ V4 sub4(const V4& a, const V4& b) {
  return V4{a.x - b.x, a.y - b.y, a.z - b.z, a.t - b.t};
}

// Triangle (P0, P1, P2) against (Q0, Q1, Q2): solve
// [P1-P0, P2-P0, Q0-Q1, Q0-Q2] (s,u,v,w)^T = Q0 - P0 by Cramer's rule; a crossing
// when det != 0 and the solution lies in both closed triangles.
__device__ __forceinline__ bool tri_tri(const V4& P0, const V4& P1, const V4& P2, const V4& Q0,
                                        const V4& Q1, const V4& Q2, double& t_out, double& x_out,
                                        double& y_out, double& z_out) {
  const V4 E1 = sub4(P1, P0);
  const V4 E2 = sub4(P2, P0);
  const V4 G1 = sub4(Q0, Q1);
  const V4 G2 = sub4(Q0, Q2);
  const V4 D = sub4(Q0, P0);
  const double det = det4(E1, E2, G1, G2);
  if (det == 0.0) return false;
  const double sn = det4(D, E2, G1, G2);
  const double un = det4(E1, D, G1, G2);
  const double vn = det4(E1, E2, D, G2);
  const double wn = det4(E1, E2, G1, D);
  bool ok;
  if (det > 0.0)
    ok = sn >= 0.0 && un >= 0.0 && (sn + un) <= det && vn >= 0.0 && wn >= 0.0 && (vn + wn) <= det;
  else
    ok = sn <= 0.0 && un <= 0.0 && (sn + un) >= det && vn <= 0.0 && wn <= 0.0 && (vn + wn) >= det;
  if (!ok) return false;
  x_out = P0.x + (sn * E1.x + un * E2.x) / det;
  y_out = P0.y + (sn * E1.y + un * E2.y) / det;
  z_out = P0.z + (sn * E1.z + un * E2.z) / det;
  t_out = P0.t + (sn * E1.t + un * E2.t) / det;
  return true;
}

}  // namespace sp
