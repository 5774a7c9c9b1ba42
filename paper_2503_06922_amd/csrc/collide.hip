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
  // a list entry's triangle and bounding sphere are loaded together, one step ahead: the next
  // entries are in flight while this lane tests the current one
  const bool mixed = d.mixed;
  const float4 no_sf = make_float4(0.f, 0.f, 0.f, -1.f);
  const double4 no_sd = make_double4(0.0, 0.0, 0.0, -1.0);
  int32_t t_nx = b0 + j < b1 ? d.cell_tris[b0 + j] : -1;
  float4 sf_nx = mixed && b0 + j < b1 ? d.cell_sf[b0 + j] : no_sf;
  double4 sd_nx = !mixed && b0 + j < b1 ? d.cell_sd[b0 + j] : no_sd;
  for (int32_t k0 = b0; k0 < b1; k0 += CL) {
    const int32_t t = t_nx;
    const float4 Sf = sf_nx;
    const double4 Sd = sd_nx;
    {
      const int32_t k2 = k0 + CL + j;
      t_nx = k2 < b1 ? d.cell_tris[k2] : -1;
      sf_nx = mixed && k2 < b1 ? d.cell_sf[k2] : no_sf;
      sd_nx = !mixed && k2 < b1 ? d.cell_sd[k2] : no_sd;
    }
    bool near;
    if (mixed) {
      const float bf = (float)band + slack;
      const float sx = pf.x - Sf.x, sy = pf.y - Sf.y, sz = pf.z - Sf.z, rr = Sf.w + bf;
      near = t >= 0 && sx * sx + sy * sy + sz * sz <= rr * rr;
    } else {
      const double sx = p.x - Sd.x, sy = p.y - Sd.y, sz = p.z - Sd.z;
      const double rr = (Sd.w + band) * (1.0 + 1e-12);
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
        d.CS[pos * N + g] = 0.0;
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
        d.CS[g] = 0.0;
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
    if (kc == K_ELEM) continue;           // contacts along the element: collide_elem_kernel
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
      d.CS[cnt * N + g] = 0.0;
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

// ---------------------------------------------------------------- contacts along elements
// Eq. 3-7 with 0 < xi < l0: the contact point on element g -> g+1 is the chord point
// p(s) = (1 - s) x_g + s x_{g+1} (N_i in the element's chord frame, where both nodes lie on the
// axis).  Per element whose two nodes are contact nodes, every triangle of the grid cells the
// chord crosses: the closest points of the chord and each of the triangle's edges (segment-
// segment, Ericson 2005, Sec. 5.1.9), the nearest edge giving s*; a candidate when 0 < s* < 1,
// the edge is not (nearly) parallel to the chord (sin^2 >= SEG_PARALLEL), p(s*) lies in front
// of the triangle, its nearest point c on the triangle is on an edge or vertex that is a
// sharp convex feature of the wall (tsharp: a fold of at least 10 degrees, a rim) and
// |p - c| <= r_c + delta.  The element's contact is the group's nearest candidate (ties to the lowest
// triangle): kind 2 at node g with s = s*, normal (p - c)/|p - c| and gap |p - c| - r_c.  A
// contact along the element that carried force at the previous iterate and is not detected
// again persists while 0 < s* < 1, p(s*) lies in front of its triangle and within the band of
// it (unless the detected one has the same normal, gap and s), as node contacts do.  The
// entries follow the node's own contacts (ordered by triangle).

// closest points of segments p1p2 and q1q2: the chord parameter s, the squared sine of their
// angle, the distance (the unconstrained minimiser clamped to [0,1]^2 one parameter at a time)
__device__ __forceinline__ double seg_closest(P3<double> p1, P3<double> p2, P3<double> q1, P3<double> q2,
                                              double* s_out, double* sin2_out) {
  const P3<double> d1 = sub(p2, p1), d2 = sub(q2, q1), r = sub(p1, q1);
  const double a = dotp(d1, d1), e = dotp(d2, d2), b = dotp(d1, d2);
  const double c = dotp(d1, r), f = dotp(d2, r);
  const double den = a * e - b * b;
  double s = den > 0.0 ? fmin(fmax((b * f - c * e) / den, 0.0), 1.0) : 0.0;
  double u = (b * s + f) / e;
  if (u < 0.0) {
    u = 0.0;
    s = fmin(fmax(-c / a, 0.0), 1.0);
  } else if (u > 1.0) {
    u = 1.0;
    s = fmin(fmax((b - c) / a, 0.0), 1.0);
  }
  *s_out = s;
  *sin2_out = den / (a * e);
  const P3<double> dd = sub(axpy(p1, s, d1), axpy(q1, u, d2));
  return sqrt(dotp(dd, dd));
}

struct ElemTest { double s, sin2, front, dist; int region, feature; P3<double> p, cp; };

// chord xa-xb against triangle t
__device__ __forceinline__ ElemTest elem_tri(const Dev& d, int64_t t, P3<double> xa, P3<double> xb) {
  const double4* rec = reinterpret_cast<const double4*>(d.tv + 12 * t);
  const double4 A = rec[0], B = rec[1], C = rec[2];
  const P3<double> a{A.x, A.y, A.z}, b{B.x, B.y, B.z}, c{C.x, C.y, C.z};
  const P3<double> nt{A.w, B.w, C.w};
  ElemTest r;
  double s1, w1, s2, w2, s3, w3;
  const double d1 = seg_closest(xa, xb, a, b, &s1, &w1);
  const double d2 = seg_closest(xa, xb, a, c, &s2, &w2);
  const double d3 = seg_closest(xa, xb, b, c, &s3, &w3);
  // the nearest edge, the first of equally near ones in the order ab, ac, bc
  r.s = s1; r.sin2 = w1;
  double dm = d1;
  if (d2 < dm) { dm = d2; r.s = s2; r.sin2 = w2; }
  if (d3 < dm) { r.s = s3; r.sin2 = w3; }
  r.p = axpy(xa, r.s, sub(xb, xa));
  r.feature = closest_feature(r.p, a, b, c, &r.cp);
  r.region = feature_region(r.feature);
  r.front = dotp(nt, sub(r.p, a));
  const P3<double> dv = sub(r.p, r.cp);
  r.dist = sqrt(dotp(dv, dv));
  return r;
}

// the chord x0-x1 meets the box [lo, hi] (slab test, widened by a relative 1e-9 so that a
// rounding never drops a cell)
__device__ __forceinline__ bool chord_meets_box(P3<double> x0, P3<double> x1, const double* lo, const double* hi) {
  double t0 = 0.0, t1 = 1.0;
  const double p0[3] = {x0.x, x0.y, x0.z}, dp[3] = {x1.x - x0.x, x1.y - x0.y, x1.z - x0.z};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double w = 1e-9 * (hi[k] - lo[k]);
    const double l = lo[k] - w, h = hi[k] + w;
    if (dp[k] == 0.0) {
      if (p0[k] < l || p0[k] > h) return false;
    } else {
      double ta = (l - p0[k]) / dp[k], tb = (h - p0[k]) / dp[k];
      if (ta > tb) { const double x = ta; ta = tb; tb = x; }
      t0 = fmax(t0, ta);
      t1 = fmin(t1, tb);
      if (t0 > t1) return false;
    }
  }
  return true;
}

template <int CL>
__global__ void __launch_bounds__(256) collide_elem_kernel(Dev d) {
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t g = gt / CL;
  const int j = (int)(gt % CL);
  if (g >= d.Ntot) return;
  const int r = d.robot_of[g];
  if (d.st_done[r]) return;
  const int64_t N = d.Ntot;
  const int64_t i = g - d.off[r], n = d.off[r + 1] - d.off[r];
  if (i == 0 || i + 1 >= n || d.n_tris == 0) return;
  if (d.guide_axis[r] >= 0) {
    // node i inside the guide (the guided nodes are the first ones, so node i + 1 may be too)
    const double s = __dadd_rn(__dmul_rn((double)i, d.l0[r]), d.depth_cur[r]);
    if (s < d.guide_len) return;
  }
  const P3<double> xa{d.X[g], d.X[N + g], d.X[2 * N + g]};
  const P3<double> xb{d.X[g + 1], d.X[N + g + 1], d.X[2 * N + g + 1]};
  const double band = d.r_c + d.delta;
  const P3<double> ab = sub(xb, xa);
  const double ab2 = dotp(ab, ab);
  // grid cells of the chord's bounding box
  int c0[3], c1[3];
  {
    const double lo[3] = {fmin(xa.x, xb.x), fmin(xa.y, xb.y), fmin(xa.z, xb.z)};
    const double hi[3] = {fmax(xa.x, xb.x), fmax(xa.y, xb.y), fmax(xa.z, xb.z)};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      c0[k] = max(0, (int)floor((lo[k] - d.g_org[k]) / d.g_h));
      c1[k] = min(d.g_dim[k] - 1, (int)floor((hi[k] - d.g_org[k]) / d.g_h));
    }
  }
  int best_t = 0x7fffffff;
  double best_d = INFINITY, best_s = 0.0;
  P3<double> best_p{0, 0, 0}, best_cp{0, 0, 0};
  for (int cz = c0[2]; cz <= c1[2]; ++cz)
    for (int cy = c0[1]; cy <= c1[1]; ++cy)
      for (int cx = c0[0]; cx <= c1[0]; ++cx) {
        const double blo[3] = {d.g_org[0] + cx * d.g_h, d.g_org[1] + cy * d.g_h, d.g_org[2] + cz * d.g_h};
        const double bhi[3] = {blo[0] + d.g_h, blo[1] + d.g_h, blo[2] + d.g_h};
        if (!chord_meets_box(xa, xb, blo, bhi)) continue;
        const int64_t cell = ((int64_t)cz * d.g_dim[1] + cy) * d.g_dim[0] + cx;
        const int32_t b0 = d.cell_start[cell], b1 = d.cell_start[cell + 1];
        for (int32_t k = b0 + j; k < b1; k += CL) {
          const int32_t t = d.cell_tris[k];
          // bounding sphere against the chord: its centre's distance to the segment
          const double4 S = d.cell_sd[k];
          const P3<double> sc{S.x, S.y, S.z};
          const double tt = ab2 > 0.0 ? fmin(fmax(dotp(sub(sc, xa), ab) / ab2, 0.0), 1.0) : 0.0;
          const P3<double> dq = sub(sc, axpy(xa, tt, ab));
          const double rr = (S.w + band) * (1.0 + 1e-12);
          if (dotp(dq, dq) > rr * rr) continue;
          const ElemTest e = elem_tri(d, t, xa, xb);
          // F_AB..F_C = 1..6: bits 0-5 of the triangle's sharp-feature mask
          const bool ok = e.sin2 >= SEG_PARALLEL && e.s > 0.0 && e.s < 1.0 && e.front > 0.0 &&
                          e.region != R_FACE && e.dist <= band &&
                          ((d.tsharp[t] >> (e.feature - 1)) & 1);
          if (ok && (e.dist < best_d || (e.dist == best_d && t < best_t))) {
            best_d = e.dist; best_t = t; best_s = e.s; best_p = e.p; best_cp = e.cp;
          }
        }
      }
  // the group's nearest candidate, ties to the lowest triangle index
  double bd = best_d;
  int bt = best_t;
#pragma unroll
  for (int o = 1; o < CL; o <<= 1) {
    const double od = __shfl_xor(bd, o);
    const int ot = __shfl_xor(bt, o);
    if (od < bd || (od == bd && ot < bt)) { bd = od; bt = ot; }
  }
  // the winning lane hands its point over to the group's first lane through registers
  const int gl = (int)(threadIdx.x & 63) & ~(CL - 1);
  const unsigned long long win = __ballot(bt != 0x7fffffff && best_t == bt && best_d == bd) &
                                 (((1ull << CL) - 1ull) << gl);
  const int wl = win ? __ffsll((long long)win) - 1 : gl;
  const double ws = __shfl(best_s, wl), wpx = __shfl(best_p.x, wl), wpy = __shfl(best_p.y, wl),
               wpz = __shfl(best_p.z, wl), wcx = __shfl(best_cp.x, wl), wcy = __shfl(best_cp.y, wl),
               wcz = __shfl(best_cp.z, wl);
  if (j != 0) return;
  int cnt = d.CC[g];
  const int base = cnt;
  auto put = [&](int32_t t, int32_t warm, double gap, double s, P3<double> nc) {
    if (cnt < MAXC) {
      d.CT[cnt * N + g] = t;
      d.CK[cnt * N + g] = K_ELEM;
      d.CW[cnt * N + g] = warm;
      d.CG[cnt * N + g] = gap;
      d.CS[cnt * N + g] = s;
      d.CN[(3 * cnt + 0) * N + g] = nc.x;
      d.CN[(3 * cnt + 1) * N + g] = nc.y;
      d.CN[(3 * cnt + 2) * N + g] = nc.z;
    }
    ++cnt;
  };
  const int64_t cb = (int64_t)r * d.cap;
  const int ncp = d.st_ncp[r];
  const bool fresh = d.st_it[r] == 0;
  int lo = 0, hi = ncp;
  while (lo < hi) {
    const int m = (lo + hi) >> 1;
    if (d.cp_node[cb + m] < i) lo = m + 1; else hi = m;
  }
  double det_gap = 0.0, det_s = 0.0;
  P3<double> det_n{0, 0, 0};
  const bool have = bt != 0x7fffffff;
  if (have) {
    int32_t warm = 0;
    for (int c = lo; c < ncp && d.cp_node[cb + c] == i; ++c)
      warm |= (d.cp_kind[cb + c] == K_ELEM && d.cp_tri[cb + c] == bt && d.cp_y[cb + c] > 0.0) ? 1 : 0;
    const double inv = 1.0 / bd;
    det_n = P3<double>{(wpx - wcx) * inv, (wpy - wcy) * inv, (wpz - wcz) * inv};
    det_gap = bd - d.r_c;
    det_s = ws;
    put(bt, warm, det_gap, det_s, det_n);
  }
  if (!fresh) {
    for (int c = lo; c < ncp && d.cp_node[cb + c] == i; ++c) {
      if (d.cp_kind[cb + c] != K_ELEM || !(d.cp_y[cb + c] > 0.0)) continue;
      const int32_t t = d.cp_tri[cb + c];
      if (have && t == bt) continue;
      const ElemTest e = elem_tri(d, t, xa, xb);
      if (!(e.s > 0.0 && e.s < 1.0 && e.front > 0.0 && e.dist > 0.0 && e.dist <= band)) continue;
      const double inv = 1.0 / e.dist;
      const P3<double> nc{(e.p.x - e.cp.x) * inv, (e.p.y - e.cp.y) * inv, (e.p.z - e.cp.z) * inv};
      const double gap = e.dist - d.r_c;
      if (have && fabs(dotp(nc, det_n) - 1.0) <= PLANE_TOL && fabs(gap - det_gap) <= PLANE_TOL &&
          fabs(e.s - det_s) <= PLANE_TOL)
        continue;
      put(t, 1, gap, e.s, nc);
    }
  }
  // order the element's entries by triangle (insertion sort of the few appended)
  const int e1 = min(cnt, MAXC);
  for (int a = base + 1; a < e1; ++a) {
    const int32_t ta = d.CT[a * N + g], wa = d.CW[a * N + g];
    const double ga = d.CG[a * N + g], sa = d.CS[a * N + g], n0 = d.CN[(3 * a) * N + g],
                 n1 = d.CN[(3 * a + 1) * N + g], n2 = d.CN[(3 * a + 2) * N + g];
    int b = a - 1;
    while (b >= base && d.CT[b * N + g] > ta) {
      d.CT[(b + 1) * N + g] = d.CT[b * N + g];
      d.CK[(b + 1) * N + g] = d.CK[b * N + g];
      d.CW[(b + 1) * N + g] = d.CW[b * N + g];
      d.CG[(b + 1) * N + g] = d.CG[b * N + g];
      d.CS[(b + 1) * N + g] = d.CS[b * N + g];
      for (int k = 0; k < 3; ++k) d.CN[(3 * (b + 1) + k) * N + g] = d.CN[(3 * b + k) * N + g];
      --b;
    }
    d.CT[(b + 1) * N + g] = ta;
    d.CK[(b + 1) * N + g] = K_ELEM;
    d.CW[(b + 1) * N + g] = wa;
    d.CG[(b + 1) * N + g] = ga;
    d.CS[(b + 1) * N + g] = sa;
    d.CN[(3 * (b + 1)) * N + g] = n0;
    d.CN[(3 * (b + 1) + 1) * N + g] = n1;
    d.CN[(3 * (b + 1) + 2) * N + g] = n2;
  }
  d.CC[g] = cnt;
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
  if (d.elements)
    hipLaunchKernelGGL(collide_elem_kernel<8>, dim3((unsigned)((d.Ntot * 8 + T - 1) / T)), dim3(T), 0, s, d);
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
