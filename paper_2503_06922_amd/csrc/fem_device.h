// Device-side data layout and small-vector math shared by the gfx950 kernels.
//
// Layout in HBM (structure of arrays, robots concatenated, node g = off[r] + i):
//   node state   X[k*Ntot + g], k = 0..6 : px py pz qw qx qy qz      (FP64)
//   rigidities   EA[g], EI[g], GJ[g]     : element g -> g+1 (the tip slot is unused)
//   out-of-bal.  F[k*Ntot + g], k = 0..5 : internal force minus actuation
//   tangent      E1[k*Ntot + g], k = 0..2: chord direction of element g -> g+1 (FP64, or
//                E1f in FP32 in mixed precision); KC[k*Ntot + g], k = 0..5: its constants
//   factor       LD[g*36 + k], LS[g*36 + k]: Cholesky blocks L[g,g] and L[g+1,g]
//   node contacts (detection output, up to MAXC per node): CC[g], CT/CK/CG/CS[s*Ntot+g],
//                CN[(3*s+d)*Ntot + g]; a contact along the element g -> g+1 is an entry of
//                node g with kind 2 and its position CS along the element
//   per-robot contact lists, solutions and Schur matrices live at per-robot
//   offsets (robot r: contacts at r*cap, right-hand sides / solutions at zoff[r]).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace accfem {

// device workspace of the wide LCP per robot (the packed factor, its diagonal, y and the
// active set by position for up to cap positions), in doubles
__host__ __device__ inline int64_t lcp_ws_doubles(int cap) {
  return (int64_t)cap * (cap + 1) / 2 + 3 * (int64_t)cap;
}
// contact kinds: a face, an edge or vertex of the wall (both at a node), along an element
enum { K_FACE = 0, K_FEAT = 1, K_ELEM = 2 };
constexpr double SEG_PARALLEL = 1e-6;  // an edge this parallel to a chord (sin^2) gives no
                                       // contact along the element
constexpr int MAXC = 48;         // contact candidates kept per node (a node in a branch
                                 // narrower than the band meets a ring of facets)
constexpr int SOLVE_THREADS = 64;  // one wavefront per robot in the solve kernel
enum { WL_ACT = 0, WL_SMALL = 1, WL_WIDE = 2, WL_BIG = 3, WL_SUB = 4, WL_N = 5 };
// Mixed precision: a robot whose residual at the last check is above this level (N, N m) has
// its element forces evaluated in FP32 with FP32 accumulation; below it, and for the
// convergence decision, in FP64 (the FP64 refinement of the Newton iteration).  FP32 forces
// carry ~1e-7 of the element forces (~1e-6 N here), far below this level.
constexpr double F32_RESIDUAL = 1e-4;

struct Dev {
  int B;
  int64_t Ntot;
  // robots
  const int64_t* off;      // [B+1]
  const int32_t* robot_of; // [Ntot]
  const double* l0;        // [B]
  const double* base_pos;  // [3B]
  const double* base_dir;  // [3B] unit
  const double* base_up;   // [3B]
  const int32_t* guide_axis;  // [B] coordinate axis of base_dir, -1 if not axis aligned
  const int32_t* solve_order; // [B] robots by decreasing number of elements
  // work lists of the current pass (rebuilt after the convergence test, in solve order): the
  // robots taking the Newton step (WL_ACT), those among them whose contact set takes the LDS
  // LCP (WL_SMALL) or the wide one (WL_WIDE), those whose wide LCP outgrew its LDS factor
  // (WL_BIG, appended by the wide LCP); lists at wl + k B, entry counts in wl_cnt[k]; the
  // substitution's items (robot | pass << 24, a robot's passes together) at wl_sub, count
  // wl_cnt[WL_SUB].  Blocks of the per-robot kernels beyond a list's count return at once.
  int32_t* wl;
  int32_t* wl_sub;
  int32_t* wl_cnt;
  // element rigidities
  double* EA;
  double* EI;
  double* GJ;
  // actuation
  int act_kind;
  int n_cables;
  double cable_radius;
  const double* cable_cos;  // [n_cables]
  const double* cable_sin;
  double* act_cur;          // [B*nv] values of each robot's current load step
  int act_nv;
  double* depth_cur;        // [B]
  double guide_len;
  // contact rule
  double r_c, delta, beta0;
  int elements;             // contacts along elements as well (kind 2)
  double newton_tol, stag_tol;
  const double* stag_r;     // [B] stagnation level per robot
  int max_newton;
  int cap;                  // contacts per robot
  // mesh
  int64_t n_tris;
  const double* tv;   // [12*T] per triangle, 32-byte aligned: a.xyz n.x, b.xyz n.y, c.xyz n.z
  const double4* tsd; // [T] bounding sphere (centroid, radius) for the FP64 screen
  const float4* tsf;  // [T] the same in FP32 (radius rounded up)
  const float4* tqf;  // [4*T] FP32 normal and vertices a, b, c for the mixed-precision screen
  const uint8_t* tsharp;  // [T] sharp convex edges (bits 0-2: ab, ac, bc) and vertices (3-5)
  // grid
  double g_org[3];
  double g_h;
  int g_dim[3];
  const int32_t* cell_start;  // [ncell+1]
  const int32_t* cell_tris;
  const double4* cell_sd;     // bounding sphere of cell_tris[k] (FP64) ...
  const float4* cell_sf;      // ... and in FP32
  // state
  double* X;
  double* F;
  double* E1;         // element chord directions (the QP tangent, see ElemK)
  float* E1f;         // mixed precision: the chord directions are stored in FP32
  const double* KC;   // [6*Ntot] per-element tangent constants a t k1 k2 k3 k4
  double* LD;
  double* LS;
  int32_t* CC;
  int32_t* CT;
  int32_t* CK;
  double* CN;
  double* CG;
  double* CS;           // kind 2: position s of the contact point along the element (else 0)
  int32_t* CW;          // entry carried force at the previous iterate (warm start of the LCP)
  // per robot contact lists (current and previous), capacity cap each
  int32_t* ct_node;   // [B*cap]
  int32_t* ct_tri;
  int32_t* ct_kind;
  double* ct_n;       // [B*cap*3]
  double* ct_gap;
  double* ct_y;
  double* ct_s;         // kind 2: row (1 - s) n on node, s n on node + 1; else s = 0
  int32_t* ct_warm;     // contact carried force at the previous iterate
  int32_t* cp_node;
  int32_t* cp_tri;
  int32_t* cp_kind;
  double* cp_n;
  double* cp_gap;
  double* cp_y;
  double* cp_s;
  // right-hand side and step: robot r owns Z[zoff[r] .. zoff[r] + 6*N_r), row 6 f + k of free
  // node f: the right-hand side b of the linear step (check_rhs_kernel), then the step dx
  const int64_t* zoff;
  double* Z;
  // forward-swept values of the right-hand-side columns (0 = b, 1 + j = contact j) at the
  // checkpoint nodes of the substitution, node-major: row 6 f + k of robot r is the zp doubles
  // at Y + (6 off[r] + 6 f + k) * zp, one per column, so that a wavefront's columns are
  // contiguous
  double* Y;
  int64_t zp;
  double* XM;         // [B*SOLVE_THREADS*6] middle node's solution of the columns swept
                      // forward inside the factorisation
  // contact products: row i of robot r is the zp doubles at W + (r*cap + i)*zp, column 0 =
  // n_i . dx_free(node of i), column 1 + j = n_i . Z_j(node of i), Z_j = K^-1 A^T e_j; then
  // the wide LCP's per-robot workspaces (lcp_ws_doubles(cap) each)
  double* W;
  double* q;          // [B*cap]
  int32_t* ac_idx;    // [B*cap] contacts with force > 0 after the LCP, in index order ...
  double* ac_y;       // ... and their forces
  // per robot iteration state
  int32_t* st_status;
  int32_t* st_done;
  int32_t* st_nc;       // current contact count
  int32_t* st_ncp;      // previous contact count
  int32_t* st_limited;  // last step limited
  int32_t* st_nlim;
  int32_t* st_nswitch;
  int32_t* st_iters;
  int32_t* st_nact;     // active contacts of the current step
  unsigned long long* st_mx;  // largest node translation of the step (bits of a double >= 0)
  int64_t* st_rhs;      // [5B] right-hand sides, those swept forward in the factorisation,
                        // passes of the substitution, contact products it forms and Newton
                        // steps with contacts, since creation / the last state reset
  double* st_rn;        // residual norm at the last check
  double* st_rnprev;
  int32_t* n_done;      // [1] robots that finished every load step of the current call
  int mixed;
  // load stepping: every robot advances through the load steps of a call on its own
  int n_steps;              // load steps of the current call
  int32_t* st_step;         // [B] current load step (1-based; 0 before the first)
  int32_t* st_it;           // [B] Newton iteration within the current load step
  int32_t* st_fin;          // [B] every load step of the call is done
  const double* act_prev;   // [B*8] ramp start (values reached by the previous call) ...
  const double* act_tgt;    // [B*8] ... and end (the call's target)
  const double* dep_prev;   // [B]
  const double* dep_tgt;    // [B]
  const double* sched_act;  // [n_steps*B*act_nv] explicit per-step values, or NULL (ramp)
  const double* sched_dep;  // [n_steps*B] explicit per-step depths, or NULL (ramp)
  double* rec_tip;          // [n_steps*B*3] tip position at the end of each load step, or NULL
  int32_t* rec_status;      // [n_steps*B] status of each load step, or NULL
  int32_t* rec_iters;       // [n_steps*B] Newton iterations of each load step, or NULL
  int32_t* steps_conv;      // [B] statistics since creation / the last state reset
  int32_t* steps_tot;
  int64_t* iters_tot;
  // QP method of the linear step: 0 exact (Schur complement + LCP), 1 ADMM (OSQP iteration)
  int qp_admm;
  double admm_rho, admm_eps;
  int admm_max_iter;
  int64_t* st_qpit;         // [B] ADMM iterations since creation / the last state reset
  // launch shapes (picked per context by the autotuner, or the defaults 8 and 256)
  int coll_lanes;           // lanes per node in contact detection: 4, 8 or 16
  int elem_block;           // threads per block of the element update: 64, 128 or 256
};

// the wide LCP's workspace of robot r (after every robot's contact products)
__device__ __forceinline__ double* lcp_ws(const Dev& d, int r) {
  return d.W + (int64_t)d.B * d.cap * d.zp + (int64_t)r * lcp_ws_doubles(d.cap);
}

// ------------------------------------------------------------------ vectors
struct V3 { double x, y, z; };
__device__ __forceinline__ V3 v3(double x, double y, double z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return V3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator*(double s, V3 a) { return V3{s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return V3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ double norm(V3 a) { return sqrt(dot(a, a)); }

// rotation matrix (row major m[3*r+c]) of a unit quaternion (w, x, y, z)
__device__ __forceinline__ void quat_to_mat(double w, double x, double y, double z, double* m) {
  m[0] = 1.0 - 2.0 * (y * y + z * z); m[1] = 2.0 * (x * y - w * z);       m[2] = 2.0 * (x * z + w * y);
  m[3] = 2.0 * (x * y + w * z);       m[4] = 1.0 - 2.0 * (x * x + z * z); m[5] = 2.0 * (y * z - w * x);
  m[6] = 2.0 * (x * z - w * y);       m[7] = 2.0 * (y * z + w * x);       m[8] = 1.0 - 2.0 * (x * x + y * y);
}

__device__ __forceinline__ V3 col(const double* m, int c) { return V3{m[c], m[3 + c], m[6 + c]}; }

// ------------------------------------------------------------------ QP tangent
// The QP tangent of eq. 20-23, K_e = Rcal K_l Rcal^T for element g -> g+1, depends only on
// the element's chord direction e1 and six constants: a = EA/l0, t = GJ/l0, k1 = 12 EI/l0^3,
// k2 = 6 EI/l0^2, k3 = 4 EI/l0, k4 = 2 EI/l0.  With equal bending stiffness about both
// section axes its 3x3 blocks are  iso(x, y) = y I + (x - y) e1 e1^T  and  skew(s) = s [e1]x.
// The element update stores e1 only (FP64, or FP32 in mixed precision, where it is
// renormalised in FP64 when read: the element matrix then stays exactly positive
// semi-definite, which rounding the assembled blocks to FP32 would not preserve); the
// kernels that need block entries generate them.
struct ElemK { double e[3]; double a, t, k1, k2, k3, k4; };

__device__ __forceinline__ ElemK load_elem(const Dev& d, int64_t g) {
  const int64_t N = d.Ntot;
  ElemK k;
  if (d.mixed) {
    const double x = d.E1f[g], y = d.E1f[N + g], z = d.E1f[2 * N + g];
    const double s = 1.0 / sqrt(x * x + y * y + z * z);
    k.e[0] = x * s; k.e[1] = y * s; k.e[2] = z * s;
  } else {
    k.e[0] = d.E1[g]; k.e[1] = d.E1[N + g]; k.e[2] = d.E1[2 * N + g];
  }
  k.a = d.KC[g]; k.t = d.KC[N + g]; k.k1 = d.KC[2 * N + g];
  k.k2 = d.KC[3 * N + g]; k.k3 = d.KC[4 * N + g]; k.k4 = d.KC[5 * N + g];
  return k;
}

// e[i] for a runtime index without dynamic register indexing
__device__ __forceinline__ double sel3(const double* e, int i) {
  return i == 0 ? e[0] : (i == 1 ? e[1] : e[2]);
}
__device__ __forceinline__ double iso_ij(int i, int j, const double* e, double x, double y) {
  return (i == j ? y : 0.0) + (x - y) * sel3(e, i) * sel3(e, j);
}
__device__ __forceinline__ double skew_ij(int i, int j, const double* e, double s) {
  // [e]x = [[0, -ez, ey], [ez, 0, -ex], [-ey, ex, 0]]
  if (i == j) return 0.0;
  const int k = 3 - i - j;                       // the remaining axis
  const double sg = ((j - i + 3) % 3 == 1) ? -1.0 : 1.0;
  return s * sg * sel3(e, k);
}

// entry (row, col), 0..5, of the element's blocks K_aa (first node), K_bb (second node)
// and K_ab (coupling, first node's rows)
__device__ __forceinline__ double k_aa(const ElemK& k, int row, int col) {
  const int I = row / 3, J = col / 3, i = row % 3, j = col % 3;
  if (I == 0 && J == 0) return iso_ij(i, j, k.e, k.a, k.k1);
  if (I == 0 && J == 1) return skew_ij(i, j, k.e, -k.k2);
  if (I == 1 && J == 0) return skew_ij(i, j, k.e, k.k2);
  return iso_ij(i, j, k.e, k.t, k.k3);
}
__device__ __forceinline__ double k_bb(const ElemK& k, int row, int col) {
  const int I = row / 3, J = col / 3, i = row % 3, j = col % 3;
  if (I == 0 && J == 0) return iso_ij(i, j, k.e, k.a, k.k1);
  if (I == 0 && J == 1) return skew_ij(i, j, k.e, k.k2);
  if (I == 1 && J == 0) return skew_ij(i, j, k.e, -k.k2);
  return iso_ij(i, j, k.e, k.t, k.k3);
}
// the node's diagonal block D (K_bb of the left element + K_aa of the right one) and its
// coupling block S = K[i, i+1] (K_ab of the right element), row-major, compile-time indices
__device__ __forceinline__ double k_ab(const ElemK& k, int row, int col);
__device__ __forceinline__ void node_blocks(const ElemK& L, const ElemK& R, bool left, bool right,
                                            double* D, double* S) {
#pragma unroll
  for (int row = 0; row < 6; ++row)
#pragma unroll
    for (int cl = 0; cl < 6; ++cl) {
      D[row * 6 + cl] = (left ? k_bb(L, row, cl) : 0.0) + (right ? k_aa(R, row, cl) : 0.0);
      S[row * 6 + cl] = right ? k_ab(R, row, cl) : 0.0;
    }
}
__device__ __forceinline__ double k_ab(const ElemK& k, int row, int col) {
  const int I = row / 3, J = col / 3, i = row % 3, j = col % 3;
  if (I == 0 && J == 0) return iso_ij(i, j, k.e, -k.a, -k.k1);
  if (I == 1 && J == 1) return iso_ij(i, j, k.e, -k.t, k.k4);
  return skew_ij(i, j, k.e, -k.k2);
}

}  // namespace accfem
