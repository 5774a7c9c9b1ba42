// Element update: internal forces and the QP tangent of the co-rotational beam
// elements, assembled node-centrically into the block-tridiagonal system.
//
// Element e = (a, b) with node positions p and triads R (from unit quaternions):
//   chord c = p_b - p_a, l = |c|, e1 = c/l; mean section y-axis q = (R_a y + R_b y)/2;
//   e3 = unit(e1 x q), e2 = e3 x e1, R_e = [e1 e2 e3]                (Battini-Pacoste frame)
//   local rotations th_a = log(R_e^T R_a), th_b = log(R_e^T R_b); stretch u = l - l0
//   generalised stresses s = K7 (th_a, u, th_b) with the Euler-Bernoulli stiffness
//   internal force = gradient of 1/2 d.K7 d through the element-frame spin and the
//   inverse left Jacobian of the log map (exact, self-equilibrated).
// The QP tangent of eq. 20-23 is the constant local stiffness turned into the
// element frame, K_e = Rcal K_l Rcal^T.  With equal bending stiffness about both
// section axes its 3x3 blocks depend on e1 only:
//   diag(x, y, y) -> y I + (x - y) e1 e1^T,   local skew blocks -> +-k2 [e1]x.
// One thread per node computes its two adjacent elements and writes the node's
// out-of-balance force F_i (6, component-major) and the diagonal block D_i and
// coupling block K[i, i+1] (6x6 each, node-major: the per-robot sweeps read them in node order).
#include "element_math.h"

namespace accfem {

struct NodeState { V3 p; double R[9]; };

__device__ __forceinline__ NodeState load_node(const Dev& d, int64_t g) {
  NodeState n;
  const int64_t N = d.Ntot;
  n.p = v3(d.X[g], d.X[N + g], d.X[2 * N + g]);
  quat_to_mat(d.X[3 * N + g], d.X[4 * N + g], d.X[5 * N + g], d.X[6 * N + g], n.R);
  return n;
}

__device__ __forceinline__ void element_force(const NodeState& A, const NodeState& Bn, double l0,
                                              double EA, double EI, double GJ, double* fa,
                                              double* fb, V3* e1_out) {
  V3T<double> e1;
  element_force_t<double>(V3T<double>{A.p.x, A.p.y, A.p.z}, A.R, V3T<double>{Bn.p.x, Bn.p.y, Bn.p.z},
                          Bn.R, l0, EA, EI, GJ, fa, fb, &e1);
  *e1_out = v3(e1.x, e1.y, e1.z);
}

// Entry (i, j) of the 3x3 blocks used by the QP tangent:
//   iso(e; x, y) = y I + (x - y) e e^T,   skew(e; s) = s [e]x
__device__ __forceinline__ double iso_ij(int i, int j, const double* e, double x, double y) {
  return (i == j ? y : 0.0) + (x - y) * e[i] * e[j];
}
__device__ __forceinline__ double skew_ij(int i, int j, const double* e, double s) {
  // [e]x = [[0, -ez, ey], [ez, 0, -ex], [-ey, ex, 0]]
  if (i == j) return 0.0;
  const int k = 3 - i - j;                       // the remaining axis
  const double sg = ((j - i + 3) % 3 == 1) ? -1.0 : 1.0;
  return s * sg * e[k];
}

struct ElemK { double e[3]; double a, t, k1, k2, k3, k4; bool on; };

__device__ __forceinline__ ElemK elem_coeffs(V3 e1, double l0, double EA, double EI, double GJ) {
  ElemK k;
  k.e[0] = e1.x; k.e[1] = e1.y; k.e[2] = e1.z;
  k.a = EA / l0; k.t = GJ / l0; k.k1 = 12.0 * EI / (l0 * l0 * l0); k.k2 = 6.0 * EI / (l0 * l0);
  k.k3 = 4.0 * EI / l0; k.k4 = 2.0 * EI / l0;
  k.on = true;
  return k;
}

__global__ void __launch_bounds__(256) elem_kernel(Dev d) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= d.Ntot) return;
  const int r = d.robot_of[g];
  if (d.st_done[r]) return;
  const int64_t o = d.off[r];
  const int64_t n = d.off[r + 1] - o;
  const int64_t i = g - o;
  const double l0 = d.l0[r];
  const int64_t N = d.Ntot;

  double F[6] = {0, 0, 0, 0, 0, 0};
  ElemK L{}, R{};
  L.on = false;
  R.on = false;
  NodeState me = load_node(d, g);
  if (i > 0) {  // element (i-1, i): this node is its end b
    NodeState A = load_node(d, g - 1);
    double fa[6], fb[6];
    V3 e1;
    element_force(A, me, l0, d.EA[g - 1], d.EI[g - 1], d.GJ[g - 1], fa, fb, &e1);
#pragma unroll
    for (int k = 0; k < 6; ++k) F[k] += fb[k];
    L = elem_coeffs(e1, l0, d.EA[g - 1], d.EI[g - 1], d.GJ[g - 1]);
  }
  if (i < n - 1) {  // element (i, i+1): this node is its end a
    NodeState Bn = load_node(d, g + 1);
    double fa[6], fb[6];
    V3 e1;
    element_force(me, Bn, l0, d.EA[g], d.EI[g], d.GJ[g], fa, fb, &e1);
#pragma unroll
    for (int k = 0; k < 6; ++k) F[k] += fa[k];
    R = elem_coeffs(e1, l0, d.EA[g], d.EI[g], d.GJ[g]);
  } else {  // tip node: subtract the actuation load (eq. 18)
    const double* v = d.act_cur + (int64_t)r * d.act_nv;
    V3 Fl = v3(0, 0, 0), Ml = v3(0, 0, 0);
    if (d.act_kind == 0) {
      for (int j = 0; j < d.n_cables; ++j) {
        // M_j = d_j x F_j with d_j = rc (0, cos, sin), F_j = -T_j e_x
        double T = v[j];
        Ml = Ml + (T * d.cable_radius) * v3(0.0, -d.cable_sin[j], d.cable_cos[j]);
      }
    } else {
      Fl = v3(v[0], v[1], v[2]);
      Ml = v3(v[3], v[4], v[5]);
    }
    V3 Fg, Mg;
    if (d.act_kind == 2) {
      Fg = Fl; Mg = Ml;
    } else {
      Fg = Fl.x * col(me.R, 0) + Fl.y * col(me.R, 1) + Fl.z * col(me.R, 2);
      Mg = Ml.x * col(me.R, 0) + Ml.y * col(me.R, 1) + Ml.z * col(me.R, 2);
    }
    F[0] -= Fg.x; F[1] -= Fg.y; F[2] -= Fg.z;
    F[3] -= Mg.x; F[4] -= Mg.y; F[5] -= Mg.z;
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) d.F[k * N + g] = F[k];
  // Diagonal block: K_bb of the left element + K_aa of the right element; coupling
  // block K[i, i+1] = K_ab of the right element.  Entries are generated as stored.
  // In mixed precision the blocks are rounded to FP32 as they are stored (the factorisation
  // upcasts them and runs in FP64; the out-of-balance force above stays FP64).
  double2* KD2 = reinterpret_cast<double2*>(d.KD + g * 36);
  double2* KS2 = reinterpret_cast<double2*>(d.KS + g * 36);
  float2* KD2f = reinterpret_cast<float2*>(d.KDf + g * 36);
  float2* KS2f = reinterpret_cast<float2*>(d.KSf + g * 36);
#pragma unroll
  for (int p = 0; p < 18; ++p) {
    double dv[2], sv[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int k = 2 * p + h, row = k / 6, cl = k % 6;
      const int I = row / 3, J = cl / 3, ii = row % 3, jj = cl % 3;
      double dd = 0.0, ss = 0.0;
      if (L.on) {
        if (I == 0 && J == 0) dd += iso_ij(ii, jj, L.e, L.a, L.k1);
        if (I == 0 && J == 1) dd += skew_ij(ii, jj, L.e, L.k2);
        if (I == 1 && J == 0) dd += skew_ij(ii, jj, L.e, -L.k2);
        if (I == 1 && J == 1) dd += iso_ij(ii, jj, L.e, L.t, L.k3);
      }
      if (R.on) {
        if (I == 0 && J == 0) { dd += iso_ij(ii, jj, R.e, R.a, R.k1); ss = iso_ij(ii, jj, R.e, -R.a, -R.k1); }
        if (I == 0 && J == 1) { dd += skew_ij(ii, jj, R.e, -R.k2); ss = skew_ij(ii, jj, R.e, -R.k2); }
        if (I == 1 && J == 0) { dd += skew_ij(ii, jj, R.e, R.k2); ss = skew_ij(ii, jj, R.e, -R.k2); }
        if (I == 1 && J == 1) { dd += iso_ij(ii, jj, R.e, R.t, R.k3); ss = iso_ij(ii, jj, R.e, -R.t, R.k4); }
      }
      dv[h] = dd;
      sv[h] = ss;
    }
    if (d.mixed) {
      KD2f[p] = make_float2((float)dv[0], (float)dv[1]);
      KS2f[p] = make_float2((float)sv[0], (float)sv[1]);
    } else {
      KD2[p] = make_double2(dv[0], dv[1]);
      KS2[p] = make_double2(sv[0], sv[1]);
    }
  }
}

void launch_elem(const Dev& d, hipStream_t s) {
  const int T = 256;
  const int64_t blocks = (d.Ntot + T - 1) / T;
  hipLaunchKernelGGL(elem_kernel, dim3((unsigned)blocks), dim3(T), 0, s, d);
}

}  // namespace accfem
