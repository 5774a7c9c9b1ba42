// Node-versus-lumen contact detection against a uniform grid of triangles.
//
// Each triangle is registered in every grid cell that its bounding box, grown by
// the detection band r_c + delta, overlaps; a node then only visits the
// triangles of its own cell (in increasing triangle index).  For each triangle
// the closest point to the node and its Voronoi region (face / edge / vertex)
// are classified as in Ericson, Real-Time Collision Detection (2005), Sec. 5.1.5,
// and the signed wall distance is s = n_t . (p - v0) with the inward normal n_t.
//   face contacts : region = face and -r_c <= s <= r_c + delta      (all of them)
//   fallback      : if a node has no face contact, the nearest edge/vertex point
//                   with s > 0 within r_c + delta (ties to the lowest triangle)
// The base node and nodes held by the insertion guide are skipped.  Results are
// written per node (up to MAXC, sorted by triangle index) and compacted per
// robot by the gather step of the solver.
// In mixed precision the per-triangle tests run in FP32 with the band widened
// by a rounding allowance, and every triangle that passes is re-tested in FP64,
// so the contact set is the FP64 one.
#include "fem_device.h"

namespace accfem {

enum { R_FACE = 0, R_EDGE = 1, R_VERT = 2 };

template <typename T>
struct P3 { T x, y, z; };
template <typename T>
__device__ __forceinline__ P3<T> sub(P3<T> a, P3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <typename T>
__device__ __forceinline__ T dotp(P3<T> a, P3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename T>
__device__ __forceinline__ P3<T> axpy(P3<T> a, T s, P3<T> b) { return {a.x + s * b.x, a.y + s * b.y, a.z + s * b.z}; }

// closest point of triangle (a, b, c) to p and its region
template <typename T>
__device__ __forceinline__ int closest_on_tri(P3<T> p, P3<T> a, P3<T> b, P3<T> c, P3<T>* out) {
  P3<T> ab = sub(b, a), ac = sub(c, a), ap = sub(p, a);
  T d1 = dotp(ab, ap), d2 = dotp(ac, ap);
  if (d1 <= T(0) && d2 <= T(0)) { *out = a; return R_VERT; }
  P3<T> bp = sub(p, b);
  T d3 = dotp(ab, bp), d4 = dotp(ac, bp);
  if (d3 >= T(0) && d4 <= d3) { *out = b; return R_VERT; }
  T vc = d1 * d4 - d3 * d2;
  if (vc <= T(0) && d1 >= T(0) && d3 <= T(0)) {
    T v = d1 / (d1 - d3);
    *out = axpy(a, v, ab);
    return R_EDGE;
  }
  P3<T> cp = sub(p, c);
  T d5 = dotp(ab, cp), d6 = dotp(ac, cp);
  if (d6 >= T(0) && d5 <= d6) { *out = c; return R_VERT; }
  T vb = d5 * d2 - d1 * d6;
  if (vb <= T(0) && d2 >= T(0) && d6 <= T(0)) {
    T w = d2 / (d2 - d6);
    *out = axpy(a, w, ac);
    return R_EDGE;
  }
  T va = d3 * d6 - d5 * d4;
  if (va <= T(0) && (d4 - d3) >= T(0) && (d5 - d6) >= T(0)) {
    T w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
    *out = axpy(b, w, sub(c, b));
    return R_EDGE;
  }
  T den = T(1) / (va + vb + vc);
  T v = vb * den, w = vc * den;
  *out = axpy(axpy(a, v, ab), w, ac);
  return R_FACE;
}

struct TriTest { int region; double s, dist; P3<double> cp; };

__device__ __forceinline__ TriTest test_tri64(const Dev& d, int64_t t, P3<double> p) {
  const int64_t T = d.n_tris;
  P3<double> a{d.tv[t], d.tv[T + t], d.tv[2 * T + t]};
  P3<double> b{d.tv[3 * T + t], d.tv[4 * T + t], d.tv[5 * T + t]};
  P3<double> c{d.tv[6 * T + t], d.tv[7 * T + t], d.tv[8 * T + t]};
  P3<double> n{d.tn[t], d.tn[T + t], d.tn[2 * T + t]};
  TriTest r;
  r.s = dotp(n, sub(p, a));
  r.region = closest_on_tri(p, a, b, c, &r.cp);
  P3<double> dv = sub(p, r.cp);
  r.dist = sqrt(dotp(dv, dv));
  return r;
}

// FP32 screen: can triangle t be a face contact or a fallback candidate?
__device__ __forceinline__ bool screen32(const Dev& d, int64_t t, P3<float> p, float band, float slack) {
  const int64_t T = d.n_tris;
  P3<float> a{d.tvf[t], d.tvf[T + t], d.tvf[2 * T + t]};
  P3<float> n{d.tnf[t], d.tnf[T + t], d.tnf[2 * T + t]};
  float s = dotp(n, sub(p, a));
  if (s < -(float)d.r_c - slack || s > band + slack) return false;
  P3<float> b{d.tvf[3 * T + t], d.tvf[4 * T + t], d.tvf[5 * T + t]};
  P3<float> c{d.tvf[6 * T + t], d.tvf[7 * T + t], d.tvf[8 * T + t]};
  P3<float> cp;
  closest_on_tri(p, a, b, c, &cp);
  P3<float> dv = sub(p, cp);
  // any FP64 candidate has s >= -r_c and lies within the band of its closest point
  return sqrtf(dotp(dv, dv)) <= band + slack;
}

__global__ void __launch_bounds__(256) collide_kernel(Dev d) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= d.Ntot) return;
  const int r = d.robot_of[g];
  if (d.st_done[r]) return;
  const int64_t N = d.Ntot;
  const int64_t i = g - d.off[r];
  int cnt = 0;
  if (i == 0 || d.n_tris == 0) { d.CC[g] = 0; return; }
  if (d.guide_axis[r] >= 0) {
    // reference arc length i*l0 + depth, without contraction (same decision as the solver)
    const double s = __dadd_rn(__dmul_rn((double)i, d.l0[r]), d.depth_cur[r]);
    if (s < d.guide_len) { d.CC[g] = 0; return; }
  }
  P3<double> p{d.X[g], d.X[N + g], d.X[2 * N + g]};
  const double band = d.r_c + d.delta;
  int cx = (int)floor((p.x - d.g_org[0]) / d.g_h);
  int cy = (int)floor((p.y - d.g_org[1]) / d.g_h);
  int cz = (int)floor((p.z - d.g_org[2]) / d.g_h);
  if (cx < 0 || cy < 0 || cz < 0 || cx >= d.g_dim[0] || cy >= d.g_dim[1] || cz >= d.g_dim[2]) {
    d.CC[g] = 0;
    return;
  }
  const int64_t cell = ((int64_t)cz * d.g_dim[1] + cy) * d.g_dim[0] + cx;
  const int32_t b0 = d.cell_start[cell], b1 = d.cell_start[cell + 1];
  int best_t = -1;
  double best_d = 0.0;
  P3<double> best_cp{0, 0, 0};
  P3<float> pf{(float)p.x, (float)p.y, (float)p.z};
  // FP32 screen allowance: coordinates ~1 m carry ~1e-7 m of rounding
  const float slack = 1e-5f;
  for (int32_t k = b0; k < b1; ++k) {
    const int64_t t = d.cell_tris[k];
    if (d.mixed && !screen32(d, t, pf, (float)band, slack)) continue;
    TriTest tt = test_tri64(d, t, p);
    if (tt.region == R_FACE) {
      if (tt.s >= -d.r_c && tt.s <= band) {
        if (cnt < MAXC) {
          d.CT[cnt * N + g] = (int32_t)t;
          d.CK[cnt * N + g] = 0;
          d.CG[cnt * N + g] = tt.s - d.r_c;
          d.CN[(3 * cnt + 0) * N + g] = d.tn[t];
          d.CN[(3 * cnt + 1) * N + g] = d.tn[d.n_tris + t];
          d.CN[(3 * cnt + 2) * N + g] = d.tn[2 * d.n_tris + t];
        }
        ++cnt;
      }
    } else if (cnt == 0 && tt.s > 0.0 && tt.dist <= band) {
      if (best_t < 0 || tt.dist < best_d) {  // cell lists are sorted: ties keep the lower index
        best_t = (int)t;
        best_d = tt.dist;
        best_cp = tt.cp;
      }
    }
  }
  if (cnt == 0 && best_t >= 0) {
    d.CT[g] = best_t;
    d.CK[g] = 1;
    d.CG[g] = best_d - d.r_c;
    double inv = 1.0 / best_d;
    d.CN[0 * N + g] = (p.x - best_cp.x) * inv;
    d.CN[1 * N + g] = (p.y - best_cp.y) * inv;
    d.CN[2 * N + g] = (p.z - best_cp.z) * inv;
    cnt = 1;
  }
  d.CC[g] = cnt;  // > MAXC flags an overflow for the gather step
}

// triangle planes: vertices to SoA, unit inward normals (FP64 and FP32 copies)
__global__ void tri_setup_kernel(const double* V, const int32_t* tri, int64_t T, double* tv,
                                 double* tn, float* tvf, float* tnf) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  double v[9];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    int32_t vi = tri[3 * t + k];
    v[3 * k] = V[3 * (int64_t)vi];
    v[3 * k + 1] = V[3 * (int64_t)vi + 1];
    v[3 * k + 2] = V[3 * (int64_t)vi + 2];
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) { tv[k * T + t] = v[k]; tvf[k * T + t] = (float)v[k]; }
  V3 e0 = v3(v[3] - v[0], v[4] - v[1], v[5] - v[2]);
  V3 e1 = v3(v[6] - v[0], v[7] - v[1], v[8] - v[2]);
  V3 n = cross(e0, e1);
  double inv = 1.0 / norm(n);
  tn[t] = n.x * inv; tn[T + t] = n.y * inv; tn[2 * T + t] = n.z * inv;
  tnf[t] = (float)(n.x * inv); tnf[T + t] = (float)(n.y * inv); tnf[2 * T + t] = (float)(n.z * inv);
}

void launch_collide(const Dev& d, hipStream_t s) {
  const int T = 256;
  const int64_t blocks = (d.Ntot + T - 1) / T;
  hipLaunchKernelGGL(collide_kernel, dim3((unsigned)blocks), dim3(T), 0, s, d);
}

void launch_tri_setup(const double* V, const int32_t* tri, int64_t T, double* tv, double* tn,
                      float* tvf, float* tnf, hipStream_t s) {
  if (T == 0) return;
  const int TB = 256;
  hipLaunchKernelGGL(tri_setup_kernel, dim3((unsigned)((T + TB - 1) / TB)), dim3(TB), 0, s, V, tri,
                     T, tv, tn, tvf, tnf);
}

}  // namespace accfem
