// Co-rotational beam element internal force, written once for a scalar type T:
// double on the Newton path, a forward-mode dual number for the exact element
// Jacobian of the adjoint (the derivative part carries one perturbation direction).
#pragma once
#include "fem_device.h"

namespace accfem {

struct Dual {
  double v, d;
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator-(Dual a) { return {-a.v, -a.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
  return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)};
}
__device__ __forceinline__ Dual operator*(double s, Dual a) { return {s * a.v, s * a.d}; }
__device__ __forceinline__ Dual operator+(double s, Dual a) { return {s + a.v, a.d}; }
__device__ __forceinline__ Dual operator-(double s, Dual a) { return {s - a.v, -a.d}; }
__device__ __forceinline__ Dual operator+(Dual a, double s) { return {a.v + s, a.d}; }
__device__ __forceinline__ Dual operator-(Dual a, double s) { return {a.v - s, a.d}; }
__device__ __forceinline__ Dual operator*(Dual a, double s) { return {a.v * s, a.d * s}; }
__device__ __forceinline__ Dual operator/(Dual a, double s) { return {a.v / s, a.d / s}; }
__device__ __forceinline__ Dual operator/(double s, Dual a) { return {s / a.v, -s * a.d / (a.v * a.v)}; }
__device__ __forceinline__ double val(double x) { return x; }
__device__ __forceinline__ double val(Dual x) { return x.v; }
__device__ __forceinline__ double tsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ Dual tsqrt(Dual x) { double s = sqrt(x.v); return {s, x.d / (2.0 * s)}; }
__device__ __forceinline__ double tcos(double x) { return cos(x); }
__device__ __forceinline__ Dual tcos(Dual x) { return {cos(x.v), -sin(x.v) * x.d}; }
__device__ __forceinline__ double tsin(double x) { return sin(x); }
__device__ __forceinline__ Dual tsin(Dual x) { return {sin(x.v), cos(x.v) * x.d}; }
__device__ __forceinline__ double tatan2(double y, double x) { return atan2(y, x); }
__device__ __forceinline__ Dual tatan2(Dual y, Dual x) {
  return {atan2(y.v, x.v), (x.v * y.d - y.v * x.d) / (x.v * x.v + y.v * y.v)};
}
__device__ __forceinline__ Dual lift(double x) { return {x, 0.0}; }

template <typename T>
struct V3T { T x, y, z; };
template <typename T>
__device__ __forceinline__ V3T<T> add(V3T<T> a, V3T<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <typename T>
__device__ __forceinline__ V3T<T> sub(V3T<T> a, V3T<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <typename T, typename S>
__device__ __forceinline__ V3T<T> scl(S s, V3T<T> a) { return {s * a.x, s * a.y, s * a.z}; }
template <typename T>
__device__ __forceinline__ T dot3(V3T<T> a, V3T<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename T>
__device__ __forceinline__ V3T<T> cross3(V3T<T> a, V3T<T> b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// theta/sin(theta) * vee(Q - Q^T)/2 : log of a rotation matrix near the identity.
// |vee(Q - Q^T)/2| = sin(theta); below 1e-3 rad theta/sin(theta) = asin(s)/s is taken
// from its series in s^2, which keeps the derivative finite at theta = 0.
template <typename T>
__device__ __forceinline__ V3T<T> so3_log(const T* Q) {
  V3T<T> v{0.5 * (Q[7] - Q[5]), 0.5 * (Q[2] - Q[6]), 0.5 * (Q[3] - Q[1])};
  T c = 0.5 * (Q[0] + Q[4] + Q[8] - 1.0);
  T s2 = dot3(v, v);
  T f;
  if (atan2(sqrt(val(s2)), val(c)) < 1e-3) {
    f = 1.0 + s2 * (1.0 / 6.0 + s2 * (3.0 / 40.0 + s2 * (5.0 / 112.0)));
  } else {
    T s = tsqrt(s2);
    f = tatan2(s, c) / s;
  }
  return scl(f, v);
}

// J_l(theta)^-T s = s + 1/2 theta x s + beta(theta) theta x (theta x s)
template <typename T>
__device__ __forceinline__ V3T<T> jl_inv_T(V3T<T> th, V3T<T> s) {
  T t2 = dot3(th, th);
  T beta;
  if (val(t2) < 1e-4) {
    beta = 1.0 / 12.0 + t2 * (1.0 / 720.0 + t2 * (1.0 / 30240.0));
  } else {
    T t = tsqrt(t2);
    beta = 1.0 / t2 - (1.0 + tcos(t)) / (2.0 * t * tsin(t));
  }
  V3T<T> ts = cross3(th, s);
  return add(add(s, scl(0.5, ts)), scl(beta, cross3(th, ts)));
}

// Internal force of element (a, b) from node positions pa, pb and triads Ra, Rb
// (row-major 3x3): fa = (force, moment) at a, fb at b; e1 = chord direction.
template <typename T>
__device__ void element_force_t(V3T<T> pa, const T* Ra, V3T<T> pb, const T* Rb, double l0,
                                double EA, double EI, double GJ, T* fa, T* fb, V3T<T>* e1_out) {
  V3T<T> c = sub(pb, pa);
  T l = tsqrt(dot3(c, c));
  V3T<T> e1 = scl(1.0 / l, c);
  V3T<T> qa{Ra[1], Ra[4], Ra[7]}, qb{Rb[1], Rb[4], Rb[7]};
  V3T<T> q = scl(0.5, add(qa, qb));
  V3T<T> r = cross3(e1, q);
  V3T<T> e3 = scl(1.0 / tsqrt(dot3(r, r)), r);
  V3T<T> e2 = cross3(e3, e1);
  T Qa[9], Qb[9];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    V3T<T> ca{Ra[j], Ra[3 + j], Ra[6 + j]}, cb{Rb[j], Rb[3 + j], Rb[6 + j]};
    Qa[j] = dot3(e1, ca); Qa[3 + j] = dot3(e2, ca); Qa[6 + j] = dot3(e3, ca);
    Qb[j] = dot3(e1, cb); Qb[3 + j] = dot3(e2, cb); Qb[6 + j] = dot3(e3, cb);
  }
  V3T<T> ta = so3_log(Qa), tb = so3_log(Qb);
  T u = l - l0;
  const double gt = GJ / l0, eb = EI / l0;
  V3T<T> sa{gt * (ta.x - tb.x), eb * (4.0 * ta.y + 2.0 * tb.y), eb * (4.0 * ta.z + 2.0 * tb.z)};
  V3T<T> sb{gt * (tb.x - ta.x), eb * (2.0 * ta.y + 4.0 * tb.y), eb * (2.0 * ta.z + 4.0 * tb.z)};
  T Nx = (EA / l0) * u;
  V3T<T> ma = jl_inv_T(ta, sa), mb = jl_inv_T(tb, sb);
  V3T<T> m = add(ma, mb);
  T q1 = dot3(q, e1), q2 = dot3(q, e2);
  V3T<T> fpb = sub(add(scl(Nx, e1), scl((m.x * q1 / q2 + m.y) / l, e3)), scl(m.z / l, e2));
  T c1 = m.x / (2.0 * q2);
  V3T<T> Ma = add(add(scl(ma.x, e1), scl(ma.y, e2)), scl(ma.z, e3));
  V3T<T> Mb = add(add(scl(mb.x, e1), scl(mb.y, e2)), scl(mb.z, e3));
  V3T<T> fta = sub(Ma, scl(c1, cross3(qa, e3)));
  V3T<T> ftb = sub(Mb, scl(c1, cross3(qb, e3)));
  fa[0] = -fpb.x; fa[1] = -fpb.y; fa[2] = -fpb.z; fa[3] = fta.x; fa[4] = fta.y; fa[5] = fta.z;
  fb[0] = fpb.x;  fb[1] = fpb.y;  fb[2] = fpb.z;  fb[3] = ftb.x; fb[4] = ftb.y; fb[5] = ftb.z;
  *e1_out = e1;
}

// Mixed-precision element force: the geometry (chord, length, stretch, element frame, the
// relative rotations R_e^T R_a, R_e^T R_b and their log maps) is formed in FP64 and cast; the
// generalised stresses, the inverse left Jacobians and the assembly of the nodal forces run in
// FP32.  Absolute coordinates are never subtracted in FP32 (a 0.6 mm element 0.6 m from the
// origin would lose 1e-4 of its strain).
struct F3 { float x, y, z; };
__device__ __forceinline__ F3 f3(V3T<double> v) { return F3{(float)v.x, (float)v.y, (float)v.z}; }
__device__ __forceinline__ F3 f3add(F3 a, F3 b) { return F3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ F3 f3sub(F3 a, F3 b) { return F3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ F3 f3scl(float s, F3 a) { return F3{s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ float f3dot(F3 a, F3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ F3 f3cross(F3 a, F3 b) {
  return F3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// J_l(theta)^-T s in FP32; beta from its series below 0.2 rad, where the closed form cancels
__device__ __forceinline__ F3 jl_inv_T_f32(F3 th, F3 s) {
  const float t2 = f3dot(th, th);
  float beta;
  if (t2 < 0.04f) {
    beta = 1.0f / 12.0f + t2 * (1.0f / 720.0f + t2 * (1.0f / 30240.0f));
  } else {
    const float t = sqrtf(t2);
    beta = 1.0f / t2 - (1.0f + cosf(t)) / (2.0f * t * sinf(t));
  }
  const F3 ts = f3cross(th, s);
  return f3add(f3add(s, f3scl(0.5f, ts)), f3scl(beta, f3cross(th, ts)));
}

__device__ inline void element_force_mixed(V3T<double> pa, const double* Ra, V3T<double> pb,
                                           const double* Rb, double l0, double EA, double EI,
                                           double GJ, float* fa, float* fb, V3T<double>* e1_out) {
  // FP64 geometry
  const V3T<double> c = sub(pb, pa);
  const double l = sqrt(dot3(c, c));
  const V3T<double> e1 = scl(1.0 / l, c);
  const V3T<double> qa{Ra[1], Ra[4], Ra[7]}, qb{Rb[1], Rb[4], Rb[7]};
  const V3T<double> q = scl(0.5, add(qa, qb));
  const V3T<double> r = cross3(e1, q);
  const V3T<double> e3 = scl(1.0 / sqrt(dot3(r, r)), r);
  const V3T<double> e2 = cross3(e3, e1);
  double Qa[9], Qb[9];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const V3T<double> ca{Ra[j], Ra[3 + j], Ra[6 + j]}, cb{Rb[j], Rb[3 + j], Rb[6 + j]};
    Qa[j] = dot3(e1, ca); Qa[3 + j] = dot3(e2, ca); Qa[6 + j] = dot3(e3, ca);
    Qb[j] = dot3(e1, cb); Qb[3 + j] = dot3(e2, cb); Qb[6 + j] = dot3(e3, cb);
  }
  const F3 ta = f3(so3_log(Qa)), tb = f3(so3_log(Qb));
  const float u = (float)(l - l0);
  const float q1 = (float)dot3(q, e1), q2 = (float)dot3(q, e2), lf = (float)l;
  const F3 E1 = f3(e1), E2 = f3(e2), E3 = f3(e3), QA = f3(qa), QB = f3(qb);
  // FP32 constitutive law and nodal forces
  const float gt = (float)(GJ / l0), eb = (float)(EI / l0), ea = (float)(EA / l0);
  const F3 sa{gt * (ta.x - tb.x), eb * (4.0f * ta.y + 2.0f * tb.y), eb * (4.0f * ta.z + 2.0f * tb.z)};
  const F3 sb{gt * (tb.x - ta.x), eb * (2.0f * ta.y + 4.0f * tb.y), eb * (2.0f * ta.z + 4.0f * tb.z)};
  const float Nx = ea * u;
  const F3 ma = jl_inv_T_f32(ta, sa), mb = jl_inv_T_f32(tb, sb);
  const F3 m = f3add(ma, mb);
  const F3 fpb = f3sub(f3add(f3scl(Nx, E1), f3scl((m.x * q1 / q2 + m.y) / lf, E3)), f3scl(m.z / lf, E2));
  const float c1 = m.x / (2.0f * q2);
  const F3 Ma = f3add(f3add(f3scl(ma.x, E1), f3scl(ma.y, E2)), f3scl(ma.z, E3));
  const F3 Mb = f3add(f3add(f3scl(mb.x, E1), f3scl(mb.y, E2)), f3scl(mb.z, E3));
  const F3 fta = f3sub(Ma, f3scl(c1, f3cross(QA, E3)));
  const F3 ftb = f3sub(Mb, f3scl(c1, f3cross(QB, E3)));
  fa[0] = -fpb.x; fa[1] = -fpb.y; fa[2] = -fpb.z; fa[3] = fta.x; fa[4] = fta.y; fa[5] = fta.z;
  fb[0] = fpb.x;  fb[1] = fpb.y;  fb[2] = fpb.z;  fb[3] = ftb.x; fb[4] = ftb.y; fb[5] = ftb.z;
  *e1_out = e1;
}

}  // namespace accfem
