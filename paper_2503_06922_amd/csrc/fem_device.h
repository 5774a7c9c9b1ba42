// Device-side data layout and small-vector math shared by the gfx950 kernels.
//
// Layout in HBM (structure of arrays, robots concatenated, node g = off[r] + i):
//   node state   X[k*Ntot + g], k = 0..6 : px py pz qw qx qy qz      (FP64)
//   rigidities   EA[g], EI[g], GJ[g]     : element g -> g+1 (the tip slot is unused)
//   out-of-bal.  F[k*Ntot + g], k = 0..5 : internal force minus actuation
//   tangent      KD[g*36 + k], k = 0..35: 6x6 diagonal block of node g (row major, node-major)
//                KS[g*36 + k]           : 6x6 block K[g, g+1]
//   factor       LD[g*36 + k], LS[g*36 + k]: Cholesky blocks L[g,g] and L[g+1,g]
//   node contacts (detection output, up to MAXC per node): CC[g], CT/CK/CG[s*Ntot+g],
//                CN[(3*s+d)*Ntot + g]
//   per-robot contact lists, solutions and Schur matrices live at per-robot
//   offsets (robot r: contacts at r*cap, right-hand sides / solutions at zoff[r]).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace accfem {

constexpr int MAXC = 8;          // contact candidates kept per node
constexpr int SOLVE_THREADS = 64;  // one wavefront per robot in the solve kernel

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
  const double* act_cur;    // [B*nv] values of the current load step
  int act_nv;
  const double* depth_cur;  // [B]
  double guide_len;
  // contact rule
  double r_c, delta, beta0;
  double newton_tol, stag_tol;
  const double* stag_r;     // [B] stagnation level per robot
  int max_newton;
  int cap;                  // contacts per robot
  // mesh
  int64_t n_tris;
  const double* tv;   // [9*T]: v0x v0y v0z v1x .. v2z, SoA (k*T + t)
  const double* tn;   // [3*T]
  const float* tvf;   // [9*T] FP32 copy for the mixed-precision prefilter
  const float* tnf;   // [3*T]
  // grid
  double g_org[3];
  double g_h;
  int g_dim[3];
  const int32_t* cell_start;  // [ncell+1]
  const int32_t* cell_tris;
  // state
  double* X;
  double* F;
  double* KD;
  double* KS;
  float* KDf;         // mixed precision: the tangent blocks are stored in FP32
  float* KSf;
  double* LD;
  double* LS;
  int32_t* CC;
  int32_t* CT;
  int32_t* CK;
  double* CN;
  double* CG;
  // per robot contact lists (current and previous), capacity cap each
  int32_t* ct_node;   // [B*cap]
  int32_t* ct_tri;
  int32_t* ct_kind;
  double* ct_n;       // [B*cap*3]
  double* ct_gap;
  double* ct_y;
  int32_t* cp_node;
  int32_t* cp_tri;
  int32_t* cp_kind;
  double* cp_n;
  double* cp_gap;
  double* cp_y;
  // solutions: robot r owns Z[zoff[r] .. zoff[r] + (1+cap)*6*N_r)
  const int64_t* zoff;
  double* Z;
  double* W;          // [B*cap*cap]
  double* q;          // [B*cap]
  // per robot iteration state
  int32_t* st_status;
  int32_t* st_done;
  int32_t* st_nc;       // current contact count
  int32_t* st_ncp;      // previous contact count
  int32_t* st_limited;  // last step limited
  int32_t* st_nlim;
  int32_t* st_nswitch;
  int32_t* st_iters;
  double* st_rn;        // residual norm at the last check
  double* st_rnprev;
  int32_t* n_done;      // [1] robots finished in this load step
  int mixed;
};

// tangent block entries (FP64, or FP32 in mixed precision, upcast for the FP64 factorisation)
__device__ __forceinline__ double kd_at(const Dev& d, int64_t idx) {
  return d.mixed ? (double)d.KDf[idx] : d.KD[idx];
}
__device__ __forceinline__ double ks_at(const Dev& d, int64_t idx) {
  return d.mixed ? (double)d.KSf[idx] : d.KS[idx];
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

}  // namespace accfem
