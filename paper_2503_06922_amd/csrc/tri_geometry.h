// Closest point of a triangle to a point and its Voronoi region (face, one of the three
// edges, one of the three vertices), after Ericson, Real-Time Collision Detection (2005),
// Sec. 5.1.5; shared by contact detection and the adjoint's constraint curvature.
#pragma once
#include "fem_device.h"

namespace accfem {

enum { R_FACE = 0, R_EDGE = 1, R_VERT = 2 };
// sub-features: 0 face, 1..3 edges ab, ac, bc, 4..6 vertices a, b, c
enum { F_FACE = 0, F_AB = 1, F_AC = 2, F_BC = 3, F_A = 4, F_B = 5, F_C = 6 };
__host__ __device__ __forceinline__ int feature_region(int f) {
  return f == F_FACE ? R_FACE : (f <= F_BC ? R_EDGE : R_VERT);
}
constexpr double PLANE_TOL = 1e-9;   // two contacts lie on the same plane (normals and gaps)

template <typename T>
struct P3 { T x, y, z; };
template <typename T>
__device__ __forceinline__ P3<T> sub(P3<T> a, P3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <typename T>
__device__ __forceinline__ T dotp(P3<T> a, P3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename T>
__device__ __forceinline__ P3<T> axpy(P3<T> a, T s, P3<T> b) { return {a.x + s * b.x, a.y + s * b.y, a.z + s * b.z}; }

// closest point of triangle (a, b, c) to p and its sub-feature (F_*)
template <typename T>
__device__ __forceinline__ int closest_feature(P3<T> p, P3<T> a, P3<T> b, P3<T> c, P3<T>* out) {
  P3<T> ab = sub(b, a), ac = sub(c, a), ap = sub(p, a);
  T d1 = dotp(ab, ap), d2 = dotp(ac, ap);
  if (d1 <= T(0) && d2 <= T(0)) { *out = a; return F_A; }
  P3<T> bp = sub(p, b);
  T d3 = dotp(ab, bp), d4 = dotp(ac, bp);
  if (d3 >= T(0) && d4 <= d3) { *out = b; return F_B; }
  T vc = d1 * d4 - d3 * d2;
  if (vc <= T(0) && d1 >= T(0) && d3 <= T(0)) {
    T v = d1 / (d1 - d3);
    *out = axpy(a, v, ab);
    return F_AB;
  }
  P3<T> cp = sub(p, c);
  T d5 = dotp(ab, cp), d6 = dotp(ac, cp);
  if (d6 >= T(0) && d5 <= d6) { *out = c; return F_C; }
  T vb = d5 * d2 - d1 * d6;
  if (vb <= T(0) && d2 >= T(0) && d6 <= T(0)) {
    T w = d2 / (d2 - d6);
    *out = axpy(a, w, ac);
    return F_AC;
  }
  T va = d3 * d6 - d5 * d4;
  if (va <= T(0) && (d4 - d3) >= T(0) && (d5 - d6) >= T(0)) {
    T w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
    *out = axpy(b, w, sub(c, b));
    return F_BC;
  }
  T den = T(1) / (va + vb + vc);
  T v = vb * den, w = vc * den;
  *out = axpy(axpy(a, v, ab), w, ac);
  return F_FACE;
}

template <typename T>
__device__ __forceinline__ int closest_on_tri(P3<T> p, P3<T> a, P3<T> b, P3<T> c, P3<T>* out) {
  return feature_region(closest_feature(p, a, b, c, out));
}

}  // namespace accfem
