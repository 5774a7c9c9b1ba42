// Adjoint gradient of a loss on node positions with respect to the actuation values,
// at a converged equilibrium of a load step (the equilibrium of eq. 19 with the
// contact conditions of eq. 12-13 and the fixed-node constraints of eq. 14-15; the
// adjoint itself is an addition to the method).
//
// At equilibrium  F(x) - F_a(x, u) - A^T y = 0  with the active contacts held
// (A_act dx = 0), base node and guided lateral DOFs fixed.  For a loss L(x) with
// gradient g the adjoint multipliers solve
//     J^T lam + A_act^T mu = g,   A_act lam = 0,      J = d(F - F_a)/dx
// and dL/du_j = lam . dF_a/du_j.  Every constraint acts on the translation of a
// single node (a contact normal, or a lateral axis of the insertion guide), so the
// KKT system is the unconstrained one in node-local bases: with an orthonormal
// basis Q_i of node i whose first k_i columns span its constraint normals,
// lam = T lam', T = blockdiag(Q_i, I), and  (T^T J^T T) lam' = T^T g  with the
// first k_i translation components of node i removed.  Dependent normals (the two
// triangles of a flat quad) fall out of the Gram-Schmidt rank test.
//
// An edge/vertex contact constrains the distance rho = |p - q| from the node to the nearest
// point q of a fixed edge line or vertex; its normal n = (p - q)/rho turns with the node,
// dn/dp = (I - n n^T - t t^T)/rho (edge of unit direction t) or (I - n n^T)/rho (vertex), so
// the contact force -y n adds -y dn/dp to the node's translation block of J.  A face
// contact is a plane and adds nothing.
//
// Kernels:
//   jac       one thread per (node, direction): exact Jacobian columns by forward-mode
//             dual numbers through the element force (material + geometric
//             stiffness) and the follower actuation load at the tip, plus the curvature of
//             the node's active edge/vertex contacts
//   basis     one thread per node: constraint basis Q_i, k_i and T^T g
//   transform one thread per node: blocks of T^T J T, fixed rows/columns removed
//   sweep     one wavefront per robot: block elimination of (T^T J T)^T from the base
//             to the tip with partial pivoting inside each 6x6 block; the tip's
//             multipliers are the last unknowns, so no back substitution is needed.
#include "element_math.h"
#include "tri_geometry.h"

namespace accfem {

namespace {

struct DualNode {
  V3T<Dual> p;
  Dual R[9];
};

__device__ __forceinline__ void node_pR(const Dev& d, int64_t g, double* p, double* R) {
  const int64_t N = d.Ntot;
  p[0] = d.X[g]; p[1] = d.X[N + g]; p[2] = d.X[2 * N + g];
  quat_to_mat(d.X[3 * N + g], d.X[4 * N + g], d.X[5 * N + g], d.X[6 * N + g], R);
}

// node state as dual numbers; direction c (0..5) seeds a translation (c < 3) or a
// spatial spin R -> exp(eps e_c^) R (c >= 3), c < 0 seeds nothing
__device__ __forceinline__ DualNode dual_node(const Dev& d, int64_t g, int c) {
  double p[3], R[9];
  node_pR(d, g, p, R);
  DualNode n;
  n.p = V3T<Dual>{lift(p[0]), lift(p[1]), lift(p[2])};
#pragma unroll
  for (int k = 0; k < 9; ++k) n.R[k] = lift(R[k]);
  if (c >= 0 && c < 3) {
    if (c == 0) n.p.x.d = 1.0;
    if (c == 1) n.p.y.d = 1.0;
    if (c == 2) n.p.z.d = 1.0;
  } else if (c >= 3) {
    const int a = c - 3;
    const double w[3] = {a == 0 ? 1.0 : 0.0, a == 1 ? 1.0 : 0.0, a == 2 ? 1.0 : 0.0};
#pragma unroll
    for (int j = 0; j < 3; ++j) {  // column j of e_a^ R = e_a x (column j of R)
      const double x = R[j], y = R[3 + j], z = R[6 + j];
      n.R[j].d = w[1] * z - w[2] * y;
      n.R[3 + j].d = w[2] * x - w[0] * z;
      n.R[6 + j].d = w[0] * y - w[1] * x;
    }
  }
  return n;
}

// dn/dp (row-major 3x3) of an edge/vertex contact of triangle t at node position p
__device__ void contact_curvature(const Dev& d, int64_t t, P3<double> p, double* H) {
  const double4* rec = reinterpret_cast<const double4*>(d.tv + 12 * t);
  const P3<double> a{rec[0].x, rec[0].y, rec[0].z}, b{rec[1].x, rec[1].y, rec[1].z},
      c{rec[2].x, rec[2].y, rec[2].z};
  P3<double> q;
  const int f = closest_feature(p, a, b, c, &q);
  const P3<double> dv = sub(p, q);
  const double rho = sqrt(dotp(dv, dv));
#pragma unroll
  for (int k = 0; k < 9; ++k) H[k] = 0.0;
  if (f == F_FACE || !(rho > 0.0)) return;
  const double n[3] = {dv.x / rho, dv.y / rho, dv.z / rho};
  double tv[3] = {0.0, 0.0, 0.0};
  if (f == F_AB || f == F_AC || f == F_BC) {
    const P3<double> e = f == F_AB ? sub(b, a) : (f == F_AC ? sub(c, a) : sub(c, b));
    const double le = sqrt(dotp(e, e));
    tv[0] = e.x / le; tv[1] = e.y / le; tv[2] = e.z / le;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      H[3 * k + j] = ((k == j ? 1.0 : 0.0) - n[k] * n[j] - tv[k] * tv[j]) / rho;
}

__global__ void __launch_bounds__(256) adj_jac_kernel(Dev d, double* JL, double* JD, double* JU) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 6 * d.Ntot) return;
  const int64_t g = t / 6;
  const int c = (int)(t % 6);
  const int r = d.robot_of[g];
  const int64_t o = d.off[r], n = d.off[r + 1] - o, i = g - o;
  const double l0 = d.l0[r];
  double col[6] = {0, 0, 0, 0, 0, 0};
  DualNode me = dual_node(d, g, c);
  if (i > 0) {  // element (i-1, i): column c of J[i-1, i] and the part of J[i, i]
    DualNode A = dual_node(d, g - 1, -1);
    Dual fa[6], fb[6];
    V3T<Dual> e1;
    element_force_t<Dual>(A.p, A.R, me.p, me.R, l0, d.EA[g - 1], d.EI[g - 1], d.GJ[g - 1], fa, fb, &e1);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      JU[(g - 1) * 36 + k * 6 + c] = fa[k].d;
      col[k] += fb[k].d;
    }
  }
  if (i < n - 1) {  // element (i, i+1): column c of J[i+1, i] and the part of J[i, i]
    DualNode Bn = dual_node(d, g + 1, -1);
    Dual fa[6], fb[6];
    V3T<Dual> e1;
    element_force_t<Dual>(me.p, me.R, Bn.p, Bn.R, l0, d.EA[g], d.EI[g], d.GJ[g], fa, fb, &e1);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      JL[(g + 1) * 36 + k * 6 + c] = fb[k].d;
      col[k] += fa[k].d;
    }
  } else if (d.act_kind != 2 && c >= 3) {
    // follower load at the tip: F_a = (R f, R m) turns with the tip triad
    const double* v = d.act_cur + (int64_t)r * d.act_nv;
    double fl[3] = {0, 0, 0}, ml[3] = {0, 0, 0};
    if (d.act_kind == 0 || d.act_kind == 3) {
      for (int j = 0; j < d.n_cables; ++j) {
        const double T = v[j] * d.cable_radius;
        ml[1] -= T * d.cable_sin[j];
        ml[2] += T * d.cable_cos[j];
        if (d.act_kind == 3) fl[0] -= v[j];
      }
    } else {
      fl[0] = v[0]; fl[1] = v[1]; fl[2] = v[2];
      ml[0] = v[3]; ml[1] = v[4]; ml[2] = v[5];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double df = 0.0, dm = 0.0;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        df += me.R[3 * k + j].d * fl[j];
        dm += me.R[3 * k + j].d * ml[j];
      }
      col[k] -= df;
      col[3 + k] -= dm;
    }
  }
  if (c < 3) {
    // curvature of the node's active edge/vertex contacts: column c of -y dn/dp
    const int64_t cb = (int64_t)r * d.cap;
    const int ncp = d.st_ncp[r];
    int lo = 0, hi = ncp;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (d.cp_node[cb + mid] < i) lo = mid + 1; else hi = mid;
    }
    const int64_t N = d.Ntot;
    const P3<double> p{d.X[g], d.X[N + g], d.X[2 * N + g]};
    for (int q = lo; q < ncp && d.cp_node[cb + q] == i; ++q) {
      const double y = d.cp_y[cb + q];
      if (!(y > 0.0) || d.cp_kind[cb + q] == 0) continue;
      double H[9];
      contact_curvature(d, d.cp_tri[cb + q], p, H);
#pragma unroll
      for (int k = 0; k < 3; ++k) col[k] -= y * H[3 * k + c];
    }
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) JD[g * 36 + k * 6 + c] = col[k];
}

// node-local constraint basis and the transformed loss gradient
__global__ void __launch_bounds__(256) adj_basis_kernel(Dev d, const int32_t* sens, int n_s,
                                                        const double* dLdp, double* QB, int32_t* KF,
                                                        double* GP) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= d.Ntot) return;
  const int r = d.robot_of[g];
  const int64_t o = d.off[r], n = d.off[r + 1] - o, i = g - o;
  double u[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  int k = 0;
  auto add_normal = [&](double nx, double ny, double nz) {
    if (k >= 3) return;
    double v[3] = {nx, ny, nz};
    for (int pass = 0; pass < 2; ++pass) {  // Gram-Schmidt, reorthogonalised once
      for (int b = 0; b < k; ++b) {
        const double s = u[b][0] * v[0] + u[b][1] * v[1] + u[b][2] * v[2];
        v[0] -= s * u[b][0]; v[1] -= s * u[b][1]; v[2] -= s * u[b][2];
      }
    }
    const double nn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    if (nn <= 1e-6) return;  // dependent on the normals already taken
    u[k][0] = v[0] / nn; u[k][1] = v[1] / nn; u[k][2] = v[2] / nn;
    ++k;
  };
  int fixed = 0;
  if (i == 0) {
    fixed = 6;
  } else {
    const int ax = d.guide_axis[r];
    if (ax >= 0 && __dadd_rn(__dmul_rn((double)i, d.l0[r]), d.depth_cur[r]) < d.guide_len) {
      for (int a = 0; a < 3; ++a)
        if (a != ax) add_normal(a == 0 ? 1.0 : 0.0, a == 1 ? 1.0 : 0.0, a == 2 ? 1.0 : 0.0);
    }
    // active contacts of this node: the robot's list is sorted by node
    const int64_t cb = (int64_t)r * d.cap;
    int lo = 0, hi = d.st_ncp[r];
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (d.cp_node[cb + mid] < i) lo = mid + 1; else hi = mid;
    }
    for (int c = lo; c < d.st_ncp[r] && d.cp_node[cb + c] == i; ++c)
      if (d.cp_y[cb + c] > 0.0 && d.cp_kind[cb + c] != K_ELEM)   // (robots with active contacts
        add_normal(d.cp_n[3 * (cb + c)], d.cp_n[3 * (cb + c) + 1],   // along an element are
                   d.cp_n[3 * (cb + c) + 2]);                        // not supported)
    fixed = k;
  }
  // complete the basis
  if (k == 0) {
    u[0][0] = 1; u[1][1] = 1; u[2][2] = 1;
  } else if (k < 3) {
    if (k == 1) {  // the coordinate axis least aligned with u0
      const double ax0 = fabs(u[0][0]), ax1 = fabs(u[0][1]), ax2 = fabs(u[0][2]);
      const int a = (ax0 <= ax1 && ax0 <= ax2) ? 0 : (ax1 <= ax2 ? 1 : 2);
      double v[3] = {a == 0 ? 1.0 : 0.0, a == 1 ? 1.0 : 0.0, a == 2 ? 1.0 : 0.0};
      const double s = u[0][a];
      v[0] -= s * u[0][0]; v[1] -= s * u[0][1]; v[2] -= s * u[0][2];
      const double nn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
      u[1][0] = v[0] / nn; u[1][1] = v[1] / nn; u[1][2] = v[2] / nn;
    }
    u[2][0] = u[0][1] * u[1][2] - u[0][2] * u[1][1];
    u[2][1] = u[0][2] * u[1][0] - u[0][0] * u[1][2];
    u[2][2] = u[0][0] * u[1][1] - u[0][1] * u[1][0];
  }
  // Q[row][col] = u[col][row]
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) QB[g * 9 + a * 3 + b] = u[b][a];
  KF[g] = fixed;
  // loss gradient of this node (translations only), turned into the basis
  double gt[3] = {0, 0, 0};
  for (int s = 0; s < n_s; ++s) {
    const int64_t si = sens[s] < 0 ? n + sens[s] : sens[s];
    if (si == i) {
      const double* p = dLdp + ((int64_t)r * n_s + s) * 3;
      gt[0] += p[0]; gt[1] += p[1]; gt[2] += p[2];
    }
  }
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const double v = u[b][0] * gt[0] + u[b][1] * gt[1] + u[b][2] * gt[2];
    GP[g * 6 + b] = (b < fixed) ? 0.0 : v;
    GP[g * 6 + 3 + b] = 0.0;
  }
}

// M <- T_a^T M T_b for a 6x6 block (row major) with T = blockdiag(Q, I), then remove the
// first ka rows and kb columns (fixed DOFs)
__device__ void transform_block(double* M, const double* Qa, const double* Qb, int ka, int kb,
                                bool diag) {
  double A[36];
#pragma unroll
  for (int k = 0; k < 36; ++k) A[k] = M[k];
  // right: columns 0..2 of every row times Qb
#pragma unroll
  for (int row = 0; row < 6; ++row) {
    double t[3];
#pragma unroll
    for (int b = 0; b < 3; ++b)
      t[b] = A[row * 6 + 0] * Qb[0 * 3 + b] + A[row * 6 + 1] * Qb[1 * 3 + b] + A[row * 6 + 2] * Qb[2 * 3 + b];
#pragma unroll
    for (int b = 0; b < 3; ++b) A[row * 6 + b] = t[b];
  }
  // left: rows 0..2 of every column times Qa^T
#pragma unroll
  for (int cl = 0; cl < 6; ++cl) {
    double t[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
      t[a] = Qa[0 * 3 + a] * A[0 * 6 + cl] + Qa[1 * 3 + a] * A[1 * 6 + cl] + Qa[2 * 3 + a] * A[2 * 6 + cl];
#pragma unroll
    for (int a = 0; a < 3; ++a) A[a * 6 + cl] = t[a];
  }
#pragma unroll
  for (int row = 0; row < 6; ++row)
#pragma unroll
    for (int cl = 0; cl < 6; ++cl) {
      double v = A[row * 6 + cl];
      if (row < ka || cl < kb) v = (diag && row == cl) ? 1.0 : 0.0;
      M[row * 6 + cl] = v;
    }
}

__global__ void __launch_bounds__(256) adj_transform_kernel(Dev d, double* JL, double* JD, double* JU,
                                                            const double* QB, const int32_t* KF) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= d.Ntot) return;
  const int r = d.robot_of[g];
  const int64_t o = d.off[r], n = d.off[r + 1] - o, i = g - o;
  double Q[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) Q[k] = QB[g * 9 + k];
  const int kf = KF[g];
  transform_block(JD + g * 36, Q, Q, kf, kf, true);
  if (i > 0) {
    double Qm[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Qm[k] = QB[(g - 1) * 9 + k];
    transform_block(JL + g * 36, Q, Qm, kf, KF[g - 1], false);
  }
  if (i < n - 1) {
    double Qp[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Qp[k] = QB[(g + 1) * 9 + k];
    transform_block(JU + g * 36, Q, Qp, kf, KF[g + 1], false);
  }
}

// v[p] <-> v[k] for a runtime p >= k (unrolled, keeps v in registers)
__device__ __forceinline__ void swap_rows(double* v, int k, int p) {
  double vk = v[k], vp = vk;
#pragma unroll
  for (int r = 0; r < 6; ++r)
    if (r == p) vp = v[r];
#pragma unroll
  for (int r = 0; r < 6; ++r)
    if (r == p) v[r] = vk;
  v[k] = vp;
}

// Forward block elimination of M = (T^T J T)^T, M[i][i-1] = J'[i-1][i]^T,
// M[i][i] = J'[i][i]^T, M[i][i+1] = J'[i+1][i]^T.  Lane j < 6 holds column j of the
// reduced diagonal block D_i, lanes 6..11 the columns of G_i = D_i^-1 M[i][i+1],
// lane 12 h_i = D_i^-1 (b_i - M[i][i-1] h_{i-1}).
__global__ void __launch_bounds__(64) adj_sweep_kernel(Dev d, const double* JL, const double* JD,
                                                       const double* JU, const double* QB,
                                                       const double* GP, double* out,
                                                       int32_t* rstat) {
  const int r = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t o = d.off[r], n = d.off[r + 1] - o;
  const int nv = d.act_nv;
  // an active contact along an element couples two nodes: not supported by this elimination
  int elem = 0;
  {
    const int64_t cb = (int64_t)r * d.cap;
    for (int c = lane; c < d.st_ncp[r]; c += 64)
      elem |= (d.cp_kind[cb + c] == K_ELEM && d.cp_y[cb + c] > 0.0) ? 1 : 0;
#pragma unroll
    for (int o2 = 32; o2 > 0; o2 >>= 1) elem |= __shfl_xor(elem, o2);
  }
  double v[6] = {0, 0, 0, 0, 0, 0};  // G_{i-1} column (lanes 6..11), h_{i-1} (lane 12)
  bool bad = false;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t g = o + i;
    // G_{i-1}[:, lane] for lanes 0..5
    double gc[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) gc[k] = __shfl(v[k], (lane < 6 ? lane + 6 : 12));
    double nv6[6];
    if (lane < 6) {
#pragma unroll
      for (int k = 0; k < 6; ++k) nv6[k] = JD[g * 36 + lane * 6 + k];
    } else if (lane < 12) {
#pragma unroll
      for (int k = 0; k < 6; ++k) nv6[k] = (i < n - 1) ? JL[(g + 1) * 36 + (lane - 6) * 6 + k] : 0.0;
    } else {
#pragma unroll
      for (int k = 0; k < 6; ++k) nv6[k] = GP[g * 6 + k];
    }
    if (i > 0 && (lane < 6 || lane == 12)) {
      // subtract M[i][i-1] * (G_{i-1}[:, lane] or h_{i-1}); M[i][i-1][row][k] = J'[i-1][i][k][row]
      const double* U = JU + (g - 1) * 36;
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const double x = gc[k];
#pragma unroll
        for (int row = 0; row < 6; ++row) nv6[row] -= U[k * 6 + row] * x;
      }
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = nv6[k];
    // Gauss-Jordan with partial pivoting on [D | M[i][i+1] | b]
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      double ck[6];
#pragma unroll
      for (int row = 0; row < 6; ++row) ck[row] = __shfl(v[row], k);
      int p = k;
      double best = fabs(ck[k]);
#pragma unroll
      for (int row = k + 1; row < 6; ++row)
        if (fabs(ck[row]) > best) { best = fabs(ck[row]); p = row; }
      swap_rows(v, k, p);
      swap_rows(ck, k, p);
      const double piv = ck[k];
      if (!(best > 0.0) || !isfinite(piv)) bad = true;
      const double tk = v[k] / piv;
#pragma unroll
      for (int row = 0; row < 6; ++row) v[row] = (row == k) ? tk : v[row] - ck[row] * tk;
    }
  }
  // lane 12 now holds the tip multipliers in the tip's basis
  if (lane == 12) {
    const int64_t gt = o + n - 1;
    double lam[6];
    const double* Q = QB + gt * 9;
#pragma unroll
    for (int a = 0; a < 3; ++a) lam[a] = Q[a * 3 + 0] * v[0] + Q[a * 3 + 1] * v[1] + Q[a * 3 + 2] * v[2];
    lam[3] = v[3]; lam[4] = v[4]; lam[5] = v[5];
    double p[3], R[9];
    node_pR(d, gt, p, R);
    const bool ok = !bad && d.st_status[r] == 0 && !elem;
    double* y = out + (int64_t)r * nv;
    if (d.act_kind == 0 || d.act_kind == 3) {
      for (int j = 0; j < d.n_cables; ++j) {
        // dF_a/dT_j = (0, R m_j), m_j = rc (0, -sin, cos); with the cable force of eq. 17
        // also (-R e_x, .)
        const double m1 = -d.cable_radius * d.cable_sin[j], m2 = d.cable_radius * d.cable_cos[j];
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) s += lam[3 + a] * (R[a * 3 + 1] * m1 + R[a * 3 + 2] * m2);
        if (d.act_kind == 3) s -= lam[0] * R[0] + lam[1] * R[3] + lam[2] * R[6];
        y[j] = ok ? s : NAN;
      }
    } else if (d.act_kind == 1) {
      // dF_a/d(f, m) = blockdiag(R, R): gradient R^T lam
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double sf = R[0 * 3 + j] * lam[0] + R[1 * 3 + j] * lam[1] + R[2 * 3 + j] * lam[2];
        const double sm = R[0 * 3 + j] * lam[3] + R[1 * 3 + j] * lam[4] + R[2 * 3 + j] * lam[5];
        y[j] = ok ? sf : NAN;
        y[3 + j] = ok ? sm : NAN;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 6; ++j) y[j] = ok ? lam[j] : NAN;
    }
    rstat[r] = bad ? 1 : (d.st_status[r] != 0 ? 2 : (elem ? 3 : 0));
  }
}

}  // namespace

void launch_adjoint(const Dev& d, const int32_t* sens, int n_s, const double* dLdp, double* JL,
                    double* JD, double* JU, double* QB, int32_t* KF, double* GP, double* out,
                    int32_t* rstat, hipStream_t s) {
  const int T = 256;
  hipLaunchKernelGGL(adj_jac_kernel, dim3((unsigned)((6 * d.Ntot + T - 1) / T)), dim3(T), 0, s, d, JL,
                     JD, JU);
  hipLaunchKernelGGL(adj_basis_kernel, dim3((unsigned)((d.Ntot + T - 1) / T)), dim3(T), 0, s, d, sens,
                     n_s, dLdp, QB, KF, GP);
  hipLaunchKernelGGL(adj_transform_kernel, dim3((unsigned)((d.Ntot + T - 1) / T)), dim3(T), 0, s, d,
                     JL, JD, JU, (const double*)QB, (const int32_t*)KF);
  hipLaunchKernelGGL(adj_sweep_kernel, dim3((unsigned)d.B), dim3(64), 0, s, d, (const double*)JL,
                     (const double*)JD, (const double*)JU, (const double*)QB, (const double*)GP, out,
                     rstat);
}

}  // namespace accfem
