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
// element frame, K_e = Rcal K_l Rcal^T; its blocks depend on the chord direction e1
// only (see ElemK), so the element update stores e1 and the solver generates the blocks.
// One thread per node computes its two adjacent elements and writes the node's
// out-of-balance force F_i (6, component-major) and the chord direction of element (i, i+1).
// Mixed precision: while the robot's residual is above F32_RESIDUAL the element forces are
// evaluated in FP32 (geometry and relative rotations formed in FP64, then cast) and
// accumulated in FP32; near convergence, and for the convergence decision, in FP64.
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
  float F32[6] = {0, 0, 0, 0, 0, 0};
  const bool f32 = d.mixed && d.st_rn[r] > F32_RESIDUAL;
  NodeState me = load_node(d, g);
  if (i > 0) {  // element (i-1, i): this node is its end b
    NodeState A = load_node(d, g - 1);
    if (f32) {
      float fa[6], fb[6];
      V3T<double> e1;
      element_force_mixed(V3T<double>{A.p.x, A.p.y, A.p.z}, A.R, V3T<double>{me.p.x, me.p.y, me.p.z},
                          me.R, l0, d.EA[g - 1], d.EI[g - 1], d.GJ[g - 1], fa, fb, &e1);
#pragma unroll
      for (int k = 0; k < 6; ++k) F32[k] += fb[k];
    } else {
      double fa[6], fb[6];
      V3 e1;
      element_force(A, me, l0, d.EA[g - 1], d.EI[g - 1], d.GJ[g - 1], fa, fb, &e1);
#pragma unroll
      for (int k = 0; k < 6; ++k) F[k] += fb[k];
    }
  }
  if (i < n - 1) {  // element (i, i+1): this node is its end a
    NodeState Bn = load_node(d, g + 1);
    V3 e1;
    if (f32) {
      float fa[6], fb[6];
      V3T<double> e;
      element_force_mixed(V3T<double>{me.p.x, me.p.y, me.p.z}, me.R, V3T<double>{Bn.p.x, Bn.p.y, Bn.p.z},
                          Bn.R, l0, d.EA[g], d.EI[g], d.GJ[g], fa, fb, &e);
      e1 = v3(e.x, e.y, e.z);
#pragma unroll
      for (int k = 0; k < 6; ++k) F32[k] += fa[k];
    } else {
      double fa[6], fb[6];
      element_force(me, Bn, l0, d.EA[g], d.EI[g], d.GJ[g], fa, fb, &e1);
#pragma unroll
      for (int k = 0; k < 6; ++k) F[k] += fa[k];
    }
    // the QP tangent of element (i, i+1) is carried by its chord direction
    if (d.mixed) {
      d.E1f[g] = (float)e1.x; d.E1f[N + g] = (float)e1.y; d.E1f[2 * N + g] = (float)e1.z;
    } else {
      d.E1[g] = e1.x; d.E1[N + g] = e1.y; d.E1[2 * N + g] = e1.z;
    }
  } else {  // tip node: subtract the actuation load (eq. 18)
    const double* v = d.act_cur + (int64_t)r * d.act_nv;
    V3 Fl = v3(0, 0, 0), Ml = v3(0, 0, 0);
    if (d.act_kind == 0 || d.act_kind == 3) {
      for (int j = 0; j < d.n_cables; ++j) {
        // M_j = d_j x F_j with d_j = rc (0, cos, sin), F_j = -T_j e_x (eq. 16)
        double T = v[j];
        Ml = Ml + (T * d.cable_radius) * v3(0.0, -d.cable_sin[j], d.cable_cos[j]);
        if (d.act_kind == 3) Fl.x -= T;  // eq. 17: the cable force itself acts on the tip
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
    if (f32) {
      F32[0] -= (float)Fg.x; F32[1] -= (float)Fg.y; F32[2] -= (float)Fg.z;
      F32[3] -= (float)Mg.x; F32[4] -= (float)Mg.y; F32[5] -= (float)Mg.z;
    } else {
      F[0] -= Fg.x; F[1] -= Fg.y; F[2] -= Fg.z;
      F[3] -= Mg.x; F[4] -= Mg.y; F[5] -= Mg.z;
    }
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) d.F[k * N + g] = f32 ? (double)F32[k] : F[k];
}

void launch_elem(const Dev& d, hipStream_t s) {
  // block size: a launch shape picked per context (autotuned or 256)
  const int T = (d.elem_block == 64 || d.elem_block == 128) ? d.elem_block : 256;
  const int64_t blocks = (d.Ntot + T - 1) / T;
  hipLaunchKernelGGL(elem_kernel, dim3((unsigned)blocks), dim3(T), 0, s, d);
}

}  // namespace accfem
