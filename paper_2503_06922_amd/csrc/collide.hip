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
//   persisting    : a contact of the previous Newton iterate with force > 0 that is not
//                   detected again (same triangle and kind) stays while the node is within
//                   r_c + delta of the triangle: a face as its plane, an edge/vertex contact
//                   as the direction from the triangle's nearest point (while s > 0), unless
//                   a detected contact at the node has the same plane (normals and gaps
//                   within PLANE_TOL)
// Every entry also carries whether it had force > 0 at the previous iterate (detected
// again with the same triangle and kind, or persisting): the LCP starts from those.  At the
// first iteration of a load step the previous iterate is the previous load step's
// equilibrium: its contacts flag the warm start but none persists.
// The base node and nodes held by the insertion guide are skipped.  Results are
// written per node (up to MAXC, ordered by kind then triangle index) and compacted
// per robot by the gather step of the solver.
// In mixed precision the per-triangle tests run in FP32 with the band widened
// by a rounding allowance, and every triangle that passes is re-tested in FP64,
// so the contact set is the FP64 one; in FP64 a bounding-sphere test rejects most
// triangles first.  The screens read packed per-triangle records (one or four
// 16-byte loads), the FP64 test the structure-of-arrays vertices.
#include "tri_geometry.h"

namespace accfem {

struct TriTest { int region; double s, dist; P3<double> cp, n; };

// tv packs a triangle as three double4: (a, n.x), (b, n.y), (c, n.z)
__device__ __forceinline__ TriTest test_tri64(const Dev& d, int64_t t, P3<double> p) {
  const double4* rec = reinterpret_cast<const double4*>(d.tv + 12 * t);
  const double4 A = rec[0], B = rec[1], C = rec[2];
  P3<double> a{A.x, A.y, A.z};
  P3<double> b{B.x, B.y, B.z};
  P3<double> c{C.x, C.y, C.z};
  TriTest r;
  r.n = P3<double>{A.w, B.w, C.w};
  r.s = dotp(r.n, sub(p, a));
  r.region = closest_on_tri(p, a, b, c, &r.cp);
  P3<double> dv = sub(p, r.cp);
  r.dist = sqrt(dotp(dv, dv));
  return r;
}

// FP32 screen: can triangle t be a face contact or a fallback candidate?  Every candidate
// lies within r_c + delta of its closest point and has s >= -r_c; after the bounding-sphere
// test of the cell walk, the plane test (s in [-r_c, r_c + delta]) is repeated in FP32,
// widened by a rounding allowance.  (A fallback candidate has s > 0 and a closest point
// within r_c + delta, so |s| <= r_c + delta holds for it too.)  tqf packs (n, a, b, c).
__device__ __forceinline__ bool screen32(const Dev& d, int64_t t, P3<float> p, float band, float slack) {
  const float4 N = d.tqf[4 * t], A = d.tqf[4 * t + 1];
  P3<float> a{A.x, A.y, A.z};
  P3<float> n{N.x, N.y, N.z};
  const float s = dotp(n, sub(p, a));
  return s >= -(float)d.r_c - slack && s <= band + slack;
}

// One group of CL lanes per node: lane j of the group takes entries j, j + CL, ... of the
// node's cell list (consecutive entries to consecutive lanes), face contacts are appended
// in ballot order, the fallback is the group's lexicographic minimum of (distance, triangle)
// (the lowest triangle index among equally near ones, as a walk in list order finds), and
// the group's first lane adds the persisting contacts and orders the node's entries.  The
// group width CL (4, 8 or 16 lanes) is a launch shape picked per context (autotuned or 8);
// the detected set does not depend on it.
template <int CL>
__global__ void __launch_bounds__(256) collide_kernel(Dev d) {
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t g = gt / CL;
  const int j = (int)(gt % CL);
  if (g >= d.Ntot) return;
  const int r = d.robot_of[g];
  if (d.st_done[r]) return;
  const int64_t N = d.Ntot;
  const int64_t i = g - d.off[r];
  if (i == 0 || d.n_tris == 0) { if (j == 0) d.CC[g] = 0; return; }
  if (d.guide_axis[r] >= 0) {
    // reference arc length i*l0 + depth, without contraction (same decision as the solver)
    const double s = __dadd_rn(__dmul_rn((double)i, d.l0[r]), d.depth_cur[r]);
    if (s < d.guide_len) { if (j == 0) d.CC[g] = 0; return; }
  }
  P3<double> p{d.X[g], d.X[N + g], d.X[2 * N + g]};
  const double band = d.r_c + d.delta;
  int cx = (int)floor((p.x - d.g_org[0]) / d.g_h);
  int cy = (int)floor((p.y - d.g_org[1]) / d.g_h);
  int cz = (int)floor((p.z - d.g_org[2]) / d.g_h);
  if (cx < 0 || cy < 0 || cz < 0 || cx >= d.g_dim[0] || cy >= d.g_dim[1] || cz >= d.g_dim[2]) {
    if (j == 0) d.CC[g] = 0;
    return;
  }
  const int64_t cell = ((int64_t)cz * d.g_dim[1] + cy) * d.g_dim[0] + cx;
  const int32_t b0 = d.cell_start[cell], b1 = d.cell_start[cell + 1];
  const int gl = (int)(threadIdx.x & 63) & ~(CL - 1);      // first lane of the group
  const unsigned long long gmask = ((1ull << CL) - 1ull) << gl;
  const unsigned long long below = (1ull << (threadIdx.x & 63)) - 1ull;
  int cnt = 0;
  int best_t = -1;
  double best_d = 0.0;
  P3<double> best_cp{0, 0, 0};
  P3<float> pf{(float)p.x, (float)p.y, (float)p.z};
  // FP32 screen allowance: coordinates ~1 m carry ~1e-7 m of rounding
  const float slack = 1e-5f;
  for (int32_t k0 = b0; k0 < b1; k0 += CL) {
    const int32_t k = k0 + j;
    const int32_t t = k < b1 ? d.cell_tris[k] : -1;
    bool near;
    if (d.mixed) {
      const float4 S = t >= 0 ? d.cell_sf[k] : make_float4(0.f, 0.f, 0.f, -1.f);
      const float bf = (float)band + slack;
      const float sx = pf.x - S.x, sy = pf.y - S.y, sz = pf.z - S.z, rr = S.w + bf;
      near = t >= 0 && sx * sx + sy * sy + sz * sz <= rr * rr;
    } else {
      const double4 S = t >= 0 ? d.cell_sd[k] : make_double4(0.0, 0.0, 0.0, -1.0);
      const double sx = p.x - S.x, sy = p.y - S.y, sz = p.z - S.z;
      const double rr = (S.w + band) * (1.0 + 1e-12);
      near = t >= 0 && sx * sx + sy * sy + sz * sz <= rr * rr;
    }
    if (near && d.mixed && !screen32(d, t, pf, (float)band, slack)) near = false;
    bool face = false;
    TriTest tt;
    if (near) {
      tt = test_tri64(d, t, p);
      if (tt.region == R_FACE) {
        face = tt.s >= -d.r_c && tt.s <= band;
      } else if (tt.s > 0.0 && tt.dist <= band) {
        if (best_t < 0 || tt.dist < best_d) {  // this lane's entries are in list order
          best_t = (int)t;
          best_d = tt.dist;
          best_cp = tt.cp;
        }
      }
    }
    const unsigned long long fm = __ballot(face) & gmask;
    if (face) {
      const int pos = cnt + __popcll(fm & below);
      if (pos < MAXC) {
        d.CT[pos * N + g] = (int32_t)t;
        d.CK[pos * N + g] = 0;
        d.CW[pos * N + g] = 0;
        d.CG[pos * N + g] = tt.s - d.r_c;
        d.CN[(3 * pos + 0) * N + g] = tt.n.x;
        d.CN[(3 * pos + 1) * N + g] = tt.n.y;
        d.CN[(3 * pos + 2) * N + g] = tt.n.z;
      }
    }
    cnt += __popcll(fm);
  }
  if (cnt == 0) {
    // the group's nearest edge/vertex candidate, ties to the lowest triangle index
    double bd = best_t >= 0 ? best_d : INFINITY;
    int bt = best_t >= 0 ? best_t : 0x7fffffff;
#pragma unroll
    for (int o = 1; o < CL; o <<= 1) {
      const double od = __shfl_xor(bd, o);
      const int ot = __shfl_xor(bt, o);
      if (od < bd || (od == bd && ot < bt)) { bd = od; bt = ot; }
    }
    if (bt != 0x7fffffff) {
      if (best_t == bt) {
        d.CT[g] = bt;
        d.CK[g] = 1;
        d.CW[g] = 0;
        d.CG[g] = best_d - d.r_c;
        const double inv = 1.0 / best_d;
        d.CN[0 * N + g] = (p.x - best_cp.x) * inv;
        d.CN[1 * N + g] = (p.y - best_cp.y) * inv;
        d.CN[2 * N + g] = (p.z - best_cp.z) * inv;
      }
      cnt = 1;
    }
  }
  __threadfence_block();                 // the group's entries precede the first lane's reads
  if (j != 0) return;
  // persisting contacts: those of this node that carried force in the previous iterate and
  // were not detected again stay while the node is within the band of their triangle,
  // unless a detected contact at the node lies on the same plane
  const int ndet = min(cnt, MAXC);
  const int64_t cb = (int64_t)r * d.cap;
  const int ncp = d.st_ncp[r];
  // first iteration of a load step: the list is the previous load step's final contacts,
  // which only flag the warm start
  const bool fresh = d.st_it[r] == 0;
  int lo = 0, hi = ncp;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (d.cp_node[cb + mid] < i) lo = mid + 1; else hi = mid;
  }
  for (int c = lo; c < ncp && d.cp_node[cb + c] == i; ++c) {
    if (!(d.cp_y[cb + c] > 0.0)) continue;
    const int32_t t = d.cp_tri[cb + c];
    const int32_t kc = d.cp_kind[cb + c];
    // detected again: it starts the LCP's active set
    bool found = false;
    for (int q = 0; q < ndet; ++q)
      if (d.CK[q * N + g] == kc && d.CT[q * N + g] == t) { d.CW[q * N + g] = 1; found = true; }
    if (found || fresh) continue;
    const TriTest tt = test_tri64(d, t, p);
    if (!(tt.dist <= band)) continue;
    // a face keeps its plane; an edge/vertex contact keeps the direction from the triangle's
    // nearest point while the node stays on the triangle's inner side
    double gap;
    P3<double> nc;
    if (kc == 0) {
      gap = tt.s - d.r_c;
      nc = tt.n;
    } else {
      if (!(tt.s > 0.0) || tt.dist == 0.0) continue;
      const double inv = 1.0 / tt.dist;
      gap = tt.dist - d.r_c;
      nc = P3<double>{(p.x - tt.cp.x) * inv, (p.y - tt.cp.y) * inv, (p.z - tt.cp.z) * inv};
    }
    bool skip = false;
    for (int q = 0; q < ndet; ++q) {
      const double nn = nc.x * d.CN[(3 * q) * N + g] + nc.y * d.CN[(3 * q + 1) * N + g] +
                        nc.z * d.CN[(3 * q + 2) * N + g];
      skip |= fabs(nn - 1.0) <= PLANE_TOL && fabs(d.CG[q * N + g] - gap) <= PLANE_TOL;
    }
    if (skip) continue;
    if (cnt < MAXC) {
      d.CT[cnt * N + g] = t;
      d.CK[cnt * N + g] = kc;
      d.CW[cnt * N + g] = 1;
      d.CG[cnt * N + g] = gap;
      d.CN[(3 * cnt + 0) * N + g] = nc.x;
      d.CN[(3 * cnt + 1) * N + g] = nc.y;
      d.CN[(3 * cnt + 2) * N + g] = nc.z;
    }
    ++cnt;
  }
  // order the node's entries by (kind, triangle): insertion sort of at most MAXC
  const int nst = min(cnt, MAXC);
  for (int a = 1; a < nst; ++a) {
    const int32_t ta = d.CT[a * N + g], ka = d.CK[a * N + g], wa = d.CW[a * N + g];
    const double ga = d.CG[a * N + g], n0 = d.CN[(3 * a) * N + g], n1 = d.CN[(3 * a + 1) * N + g],
                 n2 = d.CN[(3 * a + 2) * N + g];
    int b = a - 1;
    while (b >= 0 && (d.CK[b * N + g] > ka || (d.CK[b * N + g] == ka && d.CT[b * N + g] > ta))) {
      d.CT[(b + 1) * N + g] = d.CT[b * N + g];
      d.CK[(b + 1) * N + g] = d.CK[b * N + g];
      d.CW[(b + 1) * N + g] = d.CW[b * N + g];
      d.CG[(b + 1) * N + g] = d.CG[b * N + g];
      for (int k = 0; k < 3; ++k) d.CN[(3 * (b + 1) + k) * N + g] = d.CN[(3 * b + k) * N + g];
      --b;
    }
    d.CT[(b + 1) * N + g] = ta;
    d.CK[(b + 1) * N + g] = ka;
    d.CW[(b + 1) * N + g] = wa;
    d.CG[(b + 1) * N + g] = ga;
    d.CN[(3 * (b + 1)) * N + g] = n0;
    d.CN[(3 * (b + 1) + 1) * N + g] = n1;
    d.CN[(3 * (b + 1) + 2) * N + g] = n2;
  }
  d.CC[g] = cnt;  // > MAXC flags an overflow for the gather step
}

// triangle planes: vertices to SoA, unit inward normals (FP64 and FP32 copies)
__global__ void tri_setup_kernel(const double* V, const int32_t* tri, int64_t T, double* tv,
                                 double4* tsd, float4* tsf, float4* tqf) {
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
  V3 e0 = v3(v[3] - v[0], v[4] - v[1], v[5] - v[2]);
  V3 e1 = v3(v[6] - v[0], v[7] - v[1], v[8] - v[2]);
  V3 n = cross(e0, e1);
  double inv = 1.0 / norm(n);
  n = inv * n;
  const double nn[3] = {n.x, n.y, n.z};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    tv[12 * t + 4 * k] = v[3 * k];
    tv[12 * t + 4 * k + 1] = v[3 * k + 1];
    tv[12 * t + 4 * k + 2] = v[3 * k + 2];
    tv[12 * t + 4 * k + 3] = nn[k];
  }
  // bounding sphere about the centroid
  const V3 cc = v3((v[0] + v[3] + v[6]) / 3.0, (v[1] + v[4] + v[7]) / 3.0, (v[2] + v[5] + v[8]) / 3.0);
  double R = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) R = fmax(R, norm(v3(v[3 * k], v[3 * k + 1], v[3 * k + 2]) - cc));
  tsd[t] = make_double4(cc.x, cc.y, cc.z, R);
  // FP32 copies; the radius is rounded up so that the sphere still contains the triangle
  tsf[t] = make_float4((float)cc.x, (float)cc.y, (float)cc.z, (float)R * (1.0f + 1e-6f) + 1e-6f);
  tqf[4 * t] = make_float4((float)n.x, (float)n.y, (float)n.z, 0.0f);
#pragma unroll
  for (int k = 0; k < 3; ++k)
    tqf[4 * t + 1 + k] = make_float4((float)v[3 * k], (float)v[3 * k + 1], (float)v[3 * k + 2], 0.0f);
}

void launch_collide(const Dev& d, hipStream_t s) {
  const int T = 256;
  const int cl = (d.coll_lanes == 4 || d.coll_lanes == 16) ? d.coll_lanes : 8;
  const int64_t blocks = (d.Ntot * cl + T - 1) / T;
  if (cl == 4) hipLaunchKernelGGL(collide_kernel<4>, dim3((unsigned)blocks), dim3(T), 0, s, d);
  else if (cl == 16) hipLaunchKernelGGL(collide_kernel<16>, dim3((unsigned)blocks), dim3(T), 0, s, d);
  else hipLaunchKernelGGL(collide_kernel<8>, dim3((unsigned)blocks), dim3(T), 0, s, d);
}

__global__ void cell_spheres_kernel(const int32_t* cell_tris, int64_t n, const double4* tsd,
                                    const float4* tsf, double4* csd, float4* csf) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int32_t t = cell_tris[k];
  csd[k] = tsd[t];
  csf[k] = tsf[t];
}

void launch_cell_spheres(const int32_t* cell_tris, int64_t n, const double4* tsd, const float4* tsf,
                         double4* csd, float4* csf, hipStream_t s) {
  if (n == 0) return;
  const int TB = 256;
  hipLaunchKernelGGL(cell_spheres_kernel, dim3((unsigned)((n + TB - 1) / TB)), dim3(TB), 0, s, cell_tris,
                     n, tsd, tsf, csd, csf);
}

void launch_tri_setup(const double* V, const int32_t* tri, int64_t T, double* tv,
                      double4* tsd, float4* tsf, float4* tqf, hipStream_t s) {
  if (T == 0) return;
  const int TB = 256;
  hipLaunchKernelGGL(tri_setup_kernel, dim3((unsigned)((T + TB - 1) / TB)), dim3(TB), 0, s, V, tri,
                     T, tv, tsd, tsf, tqf);
}

}  // namespace accfem
