// Host orchestration and the C ABI (include/accfem.h): context and device
// memory, lumen upload with its uniform grid, load stepping and the Newton loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/accfem.h"
#include "fem_device.h"

namespace accfem {
void launch_elem(const Dev& d, hipStream_t s);
void launch_collide(const Dev& d, hipStream_t s);
void launch_solve_phase(const Dev& d, int phase, hipStream_t s);
void launch_lcp_small(const Dev& d, hipStream_t s);
void launch_lcp_wide(const Dev& d, hipStream_t s);
void launch_gather(const Dev& d, hipStream_t s);
void launch_adjoint(const Dev& d, const int32_t* sens, int n_s, const double* dLdp, double* JL,
                    double* JD, double* JU, double* QB, int32_t* KF, double* GP, double* out,
                    int32_t* rstat, hipStream_t s);
void launch_tri_setup(const double* V, const int32_t* tri, int64_t T, double* tv,
                      double4* tsd, float4* tsf, float4* tqf, hipStream_t s);
void launch_cell_spheres(const int32_t* cell_tris, int64_t n, const double4* tsd, const float4* tsf,
                         double4* csd, float4* csf, hipStream_t s);
void launch_lcp_check(double* W, const double* q, int m, double* y, double* scratch, int* code,
                      hipStream_t s);

// ------------------------------------------------------------------ setup kernels
// straight reference configuration S_0 and the per-element rigidities
__global__ void init_state_kernel(Dev d, double r_out, double r_in, double E, double nu,
                                  double tip_len, double shE, double shA, double shI,
                                  const double* length, double* KC) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= d.Ntot) return;
  const int r = d.robot_of[g];
  const int64_t o = d.off[r], n = d.off[r + 1] - o, i = g - o;
  const double l0 = d.l0[r];
  V3 t = v3(d.base_dir[3 * r], d.base_dir[3 * r + 1], d.base_dir[3 * r + 2]);
  V3 u = v3(d.base_up[3 * r], d.base_up[3 * r + 1], d.base_up[3 * r + 2]);
  u = u - dot(u, t) * t;
  u = (1.0 / norm(u)) * u;
  V3 b = cross(t, u);
  const int64_t N = d.Ntot;
  V3 p = v3(d.base_pos[3 * r], d.base_pos[3 * r + 1], d.base_pos[3 * r + 2]) + ((double)i * l0) * t;
  d.X[g] = p.x; d.X[N + g] = p.y; d.X[2 * N + g] = p.z;
  // quaternion of R = [t u b] (columns), Shepperd's method
  const double m00 = t.x, m01 = u.x, m02 = b.x, m10 = t.y, m11 = u.y, m12 = b.y, m20 = t.z,
               m21 = u.z, m22 = b.z;
  double w, x, y, z;
  const double tr = m00 + m11 + m22;
  if (tr > 0.0) {
    double s = 2.0 * sqrt(tr + 1.0);
    w = 0.25 * s; x = (m21 - m12) / s; y = (m02 - m20) / s; z = (m10 - m01) / s;
  } else if (m00 > m11 && m00 > m22) {
    double s = 2.0 * sqrt(1.0 + m00 - m11 - m22);
    w = (m21 - m12) / s; x = 0.25 * s; y = (m01 + m10) / s; z = (m02 + m20) / s;
  } else if (m11 > m22) {
    double s = 2.0 * sqrt(1.0 + m11 - m00 - m22);
    w = (m02 - m20) / s; x = (m01 + m10) / s; y = 0.25 * s; z = (m12 + m21) / s;
  } else {
    double s = 2.0 * sqrt(1.0 + m22 - m00 - m11);
    w = (m10 - m01) / s; x = (m02 + m20) / s; y = (m12 + m21) / s; z = 0.25 * s;
  }
  d.X[3 * N + g] = w; d.X[4 * N + g] = x; d.X[5 * N + g] = y; d.X[6 * N + g] = z;
  if (i < n - 1) {
    // tube section: A = pi (ro^2 - ri^2), I = pi/4 (ro^4 - ri^4), J = 2 I, G = E / 2(1 + nu)
    const double PI = 3.14159265358979323846;
    double A = PI * (r_out * r_out - r_in * r_in);
    double I = PI / 4.0 * (r_out * r_out * r_out * r_out - r_in * r_in * r_in * r_in);
    double Ee = E;
    const double mid = ((double)i + 0.5) * l0;
    if (tip_len > 0.0 && mid < length[r] - tip_len) { A = shA; I = shI; Ee = shE; }
    const double G = Ee / (2.0 * (1.0 + nu));
    d.EA[g] = Ee * A;
    d.EI[g] = Ee * I;
    d.GJ[g] = G * 2.0 * I;
    // constants of the QP tangent blocks (Euler-Bernoulli space-frame stiffness)
    const double EA = d.EA[g], EI = d.EI[g], GJ = d.GJ[g];
    KC[g] = EA / l0;
    KC[N + g] = GJ / l0;
    KC[2 * N + g] = 12.0 * EI / (l0 * l0 * l0);
    KC[3 * N + g] = 6.0 * EI / (l0 * l0);
    KC[4 * N + g] = 4.0 * EI / l0;
    KC[5 * N + g] = 2.0 * EI / l0;
  } else {
    for (int k = 0; k < 6; ++k) KC[k * N + g] = 0.0;
    d.E1[g] = 0.0; d.E1[N + g] = 0.0; d.E1[2 * N + g] = 0.0;
    d.E1f[g] = 0.0f; d.E1f[N + g] = 0.0f; d.E1f[2 * N + g] = 0.0f;
  }
}

// node-major 6x6 blocks of the QP tangent from the element chord directions (verification output)
__global__ void assemble_kernel(Dev d, double* KD, double* KS) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= d.Ntot) return;
  const int r = d.robot_of[g];
  const int64_t o = d.off[r], n = d.off[r + 1] - o, i = g - o;
  const bool left = i > 0, right = i < n - 1;
  const ElemK KL = load_elem(d, left ? g - 1 : g), KR = load_elem(d, right ? g : g - 1);
  for (int row = 0; row < 6; ++row)
    for (int cl = 0; cl < 6; ++cl) {
      KD[g * 36 + row * 6 + cl] = (left ? k_bb(KL, row, cl) : 0.0) + (right ? k_aa(KR, row, cl) : 0.0);
      KS[g * 36 + row * 6 + cl] = right ? k_ab(KR, row, cl) : 0.0;
    }
}

// load step j of n: interpolate actuation and depth, reset per-robot Newton state
__global__ void set_load_kernel(Dev d, const double* act_prev, const double* act_tgt,
                                double* act_cur, const double* dep_prev, const double* dep_tgt,
                                double* dep_cur, int j, int n) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= d.B) return;
  const double f = (double)j / (double)n;
  for (int k = 0; k < d.act_nv; ++k) {
    const int64_t q = (int64_t)r * d.act_nv + k;
    act_cur[q] = (j == n) ? act_tgt[q] : act_prev[q] + (act_tgt[q] - act_prev[q]) * f;
  }
  dep_cur[r] = (j == n) ? dep_tgt[r] : dep_prev[r] + (dep_tgt[r] - dep_prev[r]) * f;
  d.st_status[r] = 1;
  d.st_done[r] = 0;
  d.st_ncp[r] = 0;
  d.st_nc[r] = 0;
  d.st_limited[r] = 1;
  d.st_nlim[r] = 0;
  d.st_nswitch[r] = 0;
  d.st_iters[r] = 0;
  d.st_rnprev[r] = INFINITY;
  d.st_rn[r] = INFINITY;
}

// Every robot runs through the load steps of a call on its own: when its Newton iteration of a
// load step has ended (converged or failed), the next pass of the loop books that load step
// and starts the robot's next one, while other robots are still iterating.
__global__ void init_steps_kernel(Dev d) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= d.B) return;
  d.st_step[r] = 0;
  d.st_it[r] = 0;
  d.st_done[r] = 1;
  d.st_fin[r] = 0;
}

// load step j of robot r (1-based): actuation and depth of the step, a fresh Newton state
__device__ void begin_load_step(const Dev& d, int r, int j) {
  const int n = d.n_steps;
  const double f = (double)j / (double)n;
  for (int k = 0; k < d.act_nv; ++k) {
    const int64_t q = (int64_t)r * d.act_nv + k;
    if (d.sched_act)
      d.act_cur[q] = d.sched_act[((int64_t)(j - 1) * d.B + r) * d.act_nv + k];
    else
      d.act_cur[q] = (j == n) ? d.act_tgt[q] : d.act_prev[q] + (d.act_tgt[q] - d.act_prev[q]) * f;
  }
  if (d.sched_dep)
    d.depth_cur[r] = d.sched_dep[(int64_t)(j - 1) * d.B + r];
  else
    d.depth_cur[r] = (j == n) ? d.dep_tgt[r] : d.dep_prev[r] + (d.dep_tgt[r] - d.dep_prev[r]) * f;
  d.st_step[r] = j;
  d.st_it[r] = 0;
  d.st_status[r] = 1;
  d.st_done[r] = 0;
  // the previous load step's final contacts stay listed: at iteration 0 detection uses them
  // only to flag the LCP's warm start (no contact persists across load steps)
  d.st_nc[r] = 0;
  d.st_limited[r] = 1;
  d.st_nlim[r] = 0;
  d.st_nswitch[r] = 0;
  d.st_iters[r] = 0;
  d.st_rnprev[r] = INFINITY;
  d.st_rn[r] = INFINITY;
}

// first kernel of every pass of the loop: a robot whose load step has ended books it (counters
// and the optional per-step records) and begins its next load step, or is finished
__global__ void advance_kernel(Dev d) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= d.B) return;
  if (d.st_fin[r] || !d.st_done[r]) return;
  const int j = d.st_step[r];
  if (j > 0) {
    d.steps_tot[r] += 1;
    d.steps_conv[r] += (d.st_status[r] == 0) ? 1 : 0;
    d.iters_tot[r] += d.st_iters[r];
    const int64_t q = (int64_t)(j - 1) * d.B + r;
    if (d.rec_status) d.rec_status[q] = d.st_status[r];
    if (d.rec_iters) d.rec_iters[q] = d.st_iters[r];
    if (d.rec_tip) {
      const int64_t t = d.off[r + 1] - 1, N = d.Ntot;
      for (int k = 0; k < 3; ++k) d.rec_tip[3 * q + k] = d.X[k * N + t];
    }
  }
  if (j >= d.n_steps) {
    d.st_fin[r] = 1;
    atomicAdd(d.n_done, 1);
    return;
  }
  begin_load_step(d, r, j + 1);
}

__global__ void renorm_kernel(Dev d) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= d.Ntot) return;
  const int64_t N = d.Ntot;
  double w = d.X[3 * N + g], x = d.X[4 * N + g], y = d.X[5 * N + g], z = d.X[6 * N + g];
  double inv = 1.0 / sqrt(w * w + x * x + y * y + z * z);
  d.X[3 * N + g] = w * inv; d.X[4 * N + g] = x * inv; d.X[5 * N + g] = y * inv; d.X[6 * N + g] = z * inv;
}

// node-major [g][7] <-> SoA [k][g]
__global__ void aos_to_soa(const double* in, double* out, int64_t N, int K) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  for (int k = 0; k < K; ++k) out[k * N + g] = in[g * K + k];
}
__global__ void soa_to_aos(const double* in, double* out, int64_t N, int K) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  for (int k = 0; k < K; ++k) out[g * K + k] = in[k * N + g];
}

}  // namespace accfem

using namespace accfem;

struct fem_ctx {
  std::string err;
  int B = 0;
  int64_t Ntot = 0;
  int io_dev = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  fem_params p{};
  std::vector<int64_t> h_off;
  std::vector<double> h_len;
  std::vector<int32_t> h_nelem;
  std::vector<void*> allocs;
  Dev d{};
  int act_kind = -1;
  int act_nv = 0;
  double* act_prev = nullptr;
  double* act_tgt = nullptr;
  double* act_cur = nullptr;
  double* dep_prev = nullptr;
  double* dep_tgt = nullptr;
  double* dep_cur = nullptr;
  int32_t* steps_conv = nullptr;
  int32_t* steps_tot = nullptr;
  int64_t* iters_tot = nullptr;
  double* length_d = nullptr;
  double* kc = nullptr;   // per-element tangent constants (written once at creation)
  bool lumen_set = false;
  bool act_set = false;
  bool solved = false;  // a load step was solved since creation / the last fem_set_state
  // adjoint workspace, allocated by the first fem_grad
  double* aJL = nullptr;
  double* aJD = nullptr;
  double* aJU = nullptr;
  double* aQB = nullptr;
  int32_t* aKF = nullptr;
  double* aGP = nullptr;
  double* aout = nullptr;
  int32_t* astat = nullptr;
  int32_t* asens = nullptr;
  double* adLdp = nullptr;
  int32_t a_ns_cap = 0;
  // lumen buffers (reallocated by fem_set_lumen)
  std::vector<void*> mesh_allocs;
  // load-stepping loop: the stream it runs on when the caller gave none, the captured graph
  // of `graph_iters` passes and the Dev it was captured with
  hipStream_t own_stream = nullptr;
  // a second stream (default priority) and fork/join events: inside a captured pass the
  // element update runs beside the detection and the LDS LCP beside the wide one
  hipStream_t side_stream = nullptr;
  hipEvent_t fork_ev[4] = {nullptr, nullptr, nullptr, nullptr};
  hipGraphExec_t graph_exec = nullptr;
  Dev graph_dev{};
  int graph_iters = 0;
  int iters_per_graph = 8;  // passes per replay between host checks of the finished count
  int32_t* h_done = nullptr;  // pinned host copy of the finished count
  // device copies of an explicit schedule and per-step records (grown as needed)
  double* sched_buf = nullptr;
  int64_t sched_cap = 0;
  double* rec_buf = nullptr;
  int64_t rec_cap = 0;
  // autotuned launch shapes: measured once, at the first solve of a context created with
  // autotune = 1 (times in us: element update at 64/128/256 threads per block, detection at
  // 4/8/16 lanes per node)
  bool tuned = false;
  double tune_us[6] = {NAN, NAN, NAN, NAN, NAN, NAN};
  int32_t* tune_save = nullptr;  // [B] the done flags while the autotuner runs every robot
  // per-kernel event timing
  bool profile = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double prof_ms[7] = {0, 0, 0, 0, 0, 0, 0};
  int64_t prof_n[7] = {0, 0, 0, 0, 0, 0, 0};
};

namespace {

thread_local std::string g_create_err;

fem_status fail(fem_ctx* c, fem_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define HIP_TRY(ctx, expr)                                                          \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return fail(ctx, FEM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
fem_status dalloc(fem_ctx* c, T** ptr, size_t count, std::vector<void*>& list) {
  void* p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc(&p, count * sizeof(T));
  if (e != hipSuccess) return fail(c, FEM_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  list.push_back(p);
  *ptr = static_cast<T*>(p);
  return FEM_OK;
}

#define ALLOC(ptr, count)                                     \
  do {                                                        \
    fem_status s_ = dalloc(c, &(ptr), (size_t)(count), c->allocs); \
    if (s_ != FEM_OK) return s_;                              \
  } while (0)

fem_status copy_in(fem_ctx* c, void* dst, const void* src, size_t bytes) {
  HIP_TRY(c, hipMemcpyAsync(dst, src, bytes, c->io_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                            c->stream));
  return FEM_OK;
}

fem_status copy_out(const fem_ctx* cc, void* dst, const void* src, size_t bytes) {
  fem_ctx* c = const_cast<fem_ctx*>(cc);
  HIP_TRY(c, hipMemcpyAsync(dst, src, bytes, c->io_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return FEM_OK;
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// launch with optional HIP-event timing of kernel class k
template <typename Fn>
fem_status timed(fem_ctx* c, hipStream_t s, int k, Fn&& launch) {
  if (!c->profile) {
    launch();
    return FEM_OK;
  }
  HIP_TRY(c, hipEventRecord(c->ev0, s));
  launch();
  HIP_TRY(c, hipEventRecord(c->ev1, s));
  HIP_TRY(c, hipEventSynchronize(c->ev1));
  float ms = 0.f;
  HIP_TRY(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
  c->prof_ms[k] += ms;
  c->prof_n[k] += 1;
  return FEM_OK;
}

// Autotuner of the launch shapes of the element update (threads per block) and of contact
// detection (lanes per node): on the context's current state, with every robot active, each
// candidate is launched once to warm up, then timed three times with HIP events on the
// loop's stream; the median decides.  Both kernels only read the state and write per-node
// outputs that the next pass recomputes, and neither result depends on the shape.  It runs
// once per context, after kTunePass passes of its first long enough call (robots inserted
// and in contact: the straight reference state would favour shapes that suit no contacts),
// or at the end of the first call if that is shorter.
constexpr int64_t kTunePass = 512;
fem_status autotune(fem_ctx* c, hipStream_t s) {
  Dev& d = c->d;
  const int B = c->B;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(c, hipEventCreate(&e0));
  HIP_TRY(c, hipEventCreate(&e1));
  int32_t* saved = c->tune_save;
  HIP_TRY(c, hipMemcpyAsync(saved, d.st_done, B * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  HIP_TRY(c, hipMemsetAsync(d.st_done, 0, B * sizeof(int32_t), s));
  auto median_us = [&](auto&& launch, double* out) -> fem_status {
    launch();
    float t[3];
    for (int k = 0; k < 3; ++k) {
      HIP_TRY(c, hipEventRecord(e0, s));
      launch();
      HIP_TRY(c, hipEventRecord(e1, s));
      HIP_TRY(c, hipEventSynchronize(e1));
      HIP_TRY(c, hipEventElapsedTime(&t[k], e0, e1));
    }
    HIP_TRY(c, hipGetLastError());
    std::sort(t, t + 3);
    *out = 1e3 * t[1];
    return FEM_OK;
  };
  const int blocks[3] = {64, 128, 256}, lanes[3] = {4, 8, 16};
  int best_b = 256, best_l = 8;
  double tb = INFINITY, tl = INFINITY;
  fem_status st = FEM_OK;
  for (int k = 0; k < 3 && st == FEM_OK; ++k) {
    d.elem_block = blocks[k];
    st = median_us([&] { launch_elem(d, s); }, &c->tune_us[k]);
    if (st == FEM_OK && c->tune_us[k] < tb) { tb = c->tune_us[k]; best_b = blocks[k]; }
  }
  for (int k = 0; k < 3 && st == FEM_OK; ++k) {
    d.coll_lanes = lanes[k];
    st = median_us([&] { launch_collide(d, s); }, &c->tune_us[3 + k]);
    if (st == FEM_OK && c->tune_us[3 + k] < tl) { tl = c->tune_us[3 + k]; best_l = lanes[k]; }
  }
  d.elem_block = best_b;
  d.coll_lanes = best_l;
  HIP_TRY(c, hipMemcpyAsync(d.st_done, saved, B * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == FEM_OK) c->tuned = true;
  return st;
}

// one pass of the loop over every robot: load-step advance, element update, detection and
// the Newton step's phases.  Two pairs of launches are independent and run on two streams
// (captured as parallel branches of the graph): the element update and the detection (both
// read the state; their outputs are disjoint), and the LDS LCP and the wide LCP (disjoint
// robot lists).
void launch_pass(const Dev& d, hipStream_t s, hipStream_t side, const hipEvent_t* ev) {
  hipLaunchKernelGGL(advance_kernel, dim3(nblk(d.B, 256)), dim3(256), 0, s, d);
  (void)hipEventRecord(ev[0], s);
  (void)hipStreamWaitEvent(side, ev[0], 0);
  launch_elem(d, side);
  launch_collide(d, s);
  (void)hipEventRecord(ev[1], side);
  (void)hipStreamWaitEvent(s, ev[1], 0);
  for (int ph = 0; ph < 3; ++ph) launch_solve_phase(d, ph, s);
  if (!d.qp_admm) {
    (void)hipEventRecord(ev[2], s);
    (void)hipStreamWaitEvent(side, ev[2], 0);
    launch_lcp_small(d, side);
    launch_lcp_wide(d, s);
    (void)hipEventRecord(ev[3], side);
    (void)hipStreamWaitEvent(s, ev[3], 0);
  }
  launch_solve_phase(d, 4, s);
}

// Run the n load steps of a call: every robot advances through them on its own (a robot whose
// load step has ended starts its next one in the following pass while the others iterate).
// Passes are replayed from a captured graph of iters_per_graph passes; the host reads the
// count of finished robots between replays.  A context with profile = 1 launches every pass
// directly with HIP events around each kernel class.
fem_status run_load_steps(fem_ctx* c, int n) {
  Dev& d = c->d;
  d.n_steps = n;
  hipStream_t xs = c->stream ? c->stream : c->own_stream;
  if (!c->stream) HIP_TRY(c, hipStreamSynchronize(nullptr));
  hipLaunchKernelGGL(init_steps_kernel, dim3(nblk(d.B, 256)), dim3(256), 0, xs, d);
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipMemsetAsync(d.n_done, 0, sizeof(int32_t), xs));
  // each load step takes at most max_newton + 1 passes, and one more books the last
  const int64_t max_pass = (int64_t)n * (c->p.max_newton + 1) + 1;
  int64_t pass = 0;
  if (c->profile) {
    for (;;) {
      fem_status s;
      if ((s = timed(c, xs, 2, [&] {
             hipLaunchKernelGGL(advance_kernel, dim3(nblk(d.B, 256)), dim3(256), 0, xs, d);
           })) != FEM_OK)
        return s;
      if ((s = timed(c, xs, 0, [&] { launch_elem(d, xs); })) != FEM_OK) return s;
      if ((s = timed(c, xs, 1, [&] { launch_collide(d, xs); })) != FEM_OK) return s;
      for (int ph = 0; ph < 5; ++ph)
        if ((s = timed(c, xs, 2 + ph, [&] { launch_solve_phase(d, ph, xs); })) != FEM_OK) return s;
      HIP_TRY(c, hipGetLastError());
      ++pass;
      HIP_TRY(c, hipMemcpyAsync(c->h_done, d.n_done, sizeof(int32_t), hipMemcpyDeviceToHost, xs));
      HIP_TRY(c, hipStreamSynchronize(xs));
      if (c->p.autotune && !c->tuned && (pass == kTunePass || *c->h_done >= d.B)) {
        fem_status s = autotune(c, xs);
        if (s != FEM_OK) return s;
      }
      if (*c->h_done >= d.B) break;
      if (pass > max_pass) return fail(c, FEM_E_HIP, "load stepping did not terminate");
    }
    return FEM_OK;
  }
  const int K = c->iters_per_graph;
  for (;;) {
    // (re)capture when the launch parameters changed (first call, new schedule, tuned shapes)
    if (!c->graph_exec || c->graph_iters != K || std::memcmp(&c->graph_dev, &d, sizeof(Dev)) != 0) {
      if (c->graph_exec) {
        HIP_TRY(c, hipGraphExecDestroy(c->graph_exec));
        c->graph_exec = nullptr;
      }
      hipGraph_t g = nullptr;
      HIP_TRY(c, hipStreamBeginCapture(xs, hipStreamCaptureModeThreadLocal));
      for (int k = 0; k < K; ++k) launch_pass(d, xs, c->side_stream, c->fork_ev);
      hipError_t e = hipStreamEndCapture(xs, &g);
      if (e != hipSuccess) return fail(c, FEM_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
      e = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        c->graph_exec = nullptr;
        return fail(c, FEM_E_HIP, std::string("graph instantiation: ") + hipGetErrorString(e));
      }
      std::memcpy(&c->graph_dev, &d, sizeof(Dev));
      c->graph_iters = K;
    }
    HIP_TRY(c, hipGraphLaunch(c->graph_exec, xs));
    pass += K;
    HIP_TRY(c, hipMemcpyAsync(c->h_done, d.n_done, sizeof(int32_t), hipMemcpyDeviceToHost, xs));
    HIP_TRY(c, hipStreamSynchronize(xs));
    if (c->p.autotune && !c->tuned && (pass >= kTunePass || *c->h_done >= d.B)) {
      fem_status s = autotune(c, xs);
      if (s != FEM_OK) return s;
    }
    if (*c->h_done >= d.B) break;
    if (pass > max_pass + K) return fail(c, FEM_E_HIP, "load stepping did not terminate");
  }
  return FEM_OK;
}

}  // namespace

extern "C" {

const char* fem_last_error(const fem_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

int64_t fem_total_nodes(const fem_ctx* c) { return c ? c->Ntot : -1; }

fem_status fem_tuning(const fem_ctx* c, int32_t* elem_block, int32_t* detect_lanes, double* times_us) {
  if (!c) return FEM_E_INVAL;
  if (elem_block) *elem_block = c->d.elem_block;
  if (detect_lanes) *detect_lanes = c->d.coll_lanes;
  if (times_us)
    for (int k = 0; k < 6; ++k) times_us[k] = c->tune_us[k];
  return FEM_OK;
}

void fem_destroy(fem_ctx* c) {
  if (!c) return;
  hipSetDevice(c->device);
  if (c->stream) hipStreamSynchronize(c->stream);
  for (void* p : c->mesh_allocs) hipFree(p);
  for (void* p : c->allocs) hipFree(p);
  if (c->own_stream) hipStreamSynchronize(c->own_stream);
  if (c->graph_exec) hipGraphExecDestroy(c->graph_exec);
  if (c->own_stream) hipStreamDestroy(c->own_stream);
  if (c->side_stream) hipStreamDestroy(c->side_stream);
  for (hipEvent_t e : c->fork_ev)
    if (e) hipEventDestroy(e);
  if (c->h_done) hipHostFree(c->h_done);
  if (c->sched_buf) hipFree(c->sched_buf);
  if (c->rec_buf) hipFree(c->rec_buf);
  if (c->ev0) hipEventDestroy(c->ev0);
  if (c->ev1) hipEventDestroy(c->ev1);
  delete c;
}

static fem_status create_impl(fem_ctx* c, const fem_params* p);

fem_status fem_create(const fem_params* p, fem_ctx** out) {
  g_create_err.clear();
  if (!p || !out) { g_create_err = "NULL params or out"; return FEM_E_INVAL; }
  *out = nullptr;
  fem_ctx* c = new fem_ctx();
  fem_status s = create_impl(c, p);
  if (s != FEM_OK) {
    g_create_err = c->err;
    fem_destroy(c);
    return s;
  }
  *out = c;
  return FEM_OK;
}

static fem_status create_impl(fem_ctx* c, const fem_params* p) {
  auto bad = [&](const std::string& m) { return fail(c, FEM_E_INVAL, m); };
  if (p->n_robots < 1 || !p->n_elem || !p->length || !p->base_pos || !p->base_dir || !p->base_up)
    return bad("n_robots < 1 or NULL robot arrays");
  if (!(p->r_out > p->r_in) || !(p->r_in >= 0.0) || !(p->E > 0.0) || !(p->nu > -1.0 && p->nu < 0.5))
    return bad("section or material out of range");
  if (p->tip_len > 0.0 && !(p->shaft_E > 0.0 && p->shaft_A > 0.0 && p->shaft_I > 0.0))
    return bad("shaft material out of range");
  if (p->n_cables < 1 || p->n_cables > 8 || !p->cable_angle) return bad("n_cables must be 1..8");
  if (!(p->contact_radius >= 0.0) || !(p->contact_margin > 0.0) || !(p->beta0 > 0.0))
    return bad("contact radius, margin or beta0 out of range");
  if (p->max_newton < 1 || p->contact_capacity < 1 || p->contact_capacity > 1024)
    return bad("max_newton or contact_capacity out of range");
  if (!(p->newton_tol > 0.0) || !(p->stag_tol >= 0.0)) return bad("tolerances out of range");
  if (p->qp_solver != FEM_QP_EXACT && p->qp_solver != FEM_QP_ADMM) return bad("unknown qp_solver");
  if (p->contact_along_elements != 0 && p->contact_along_elements != 1)
    return bad("contact_along_elements must be 0 or 1");
  if (p->contact_along_elements && p->qp_solver != FEM_QP_EXACT)
    return bad("contacts along elements need qp_solver = FEM_QP_EXACT");
  if (p->admm_rho < 0.0 || p->admm_eps < 0.0 || p->admm_max_iter < 0)
    return bad("ADMM parameters out of range");
  c->p = *p;
  c->B = p->n_robots;
  c->io_dev = p->io_on_device ? 1 : 0;
  c->stream = (hipStream_t)p->hip_stream;
  hipGetDevice(&c->device);
  c->h_off.assign(c->B + 1, 0);
  c->h_nelem.assign(p->n_elem, p->n_elem + c->B);
  c->h_len.assign(p->length, p->length + c->B);
  std::vector<double> bp(p->base_pos, p->base_pos + 3 * c->B), bd(3 * c->B), bu(p->base_up, p->base_up + 3 * c->B);
  std::vector<int32_t> gaxis(c->B, -1);
  std::vector<double> l0(c->B), stag(c->B);
  for (int r = 0; r < c->B; ++r) {
    if (c->h_nelem[r] < 1 || !(c->h_len[r] > 0.0)) return bad("n_elem < 1 or length <= 0");
    c->h_off[r + 1] = c->h_off[r] + c->h_nelem[r] + 1;
    l0[r] = c->h_len[r] / c->h_nelem[r];
    {
      // stagnation level: stag_tol raised to ten times the rounding floor of the
      // out-of-balance force, eps * max(EA)/l0 * (1 m) * sqrt(DOFs)
      const double PI = 3.14159265358979323846;
      double ea = p->E * PI * (p->r_out * p->r_out - p->r_in * p->r_in);
      bool shaft = false;
      if (p->tip_len > 0.0)
        for (int e = 0; e < c->h_nelem[r] && !shaft; ++e)
          shaft = ((double)e + 0.5) * l0[r] < c->h_len[r] - p->tip_len;
      if (shaft) ea = std::max(ea, p->shaft_E * p->shaft_A);
      const double floor_r = 2.220446049250313e-16 * ea / l0[r] * std::sqrt(6.0 * (c->h_nelem[r] + 1));
      stag[r] = std::max(p->stag_tol, 10.0 * floor_r);
    }
    double nn = std::sqrt(p->base_dir[3 * r] * p->base_dir[3 * r] + p->base_dir[3 * r + 1] * p->base_dir[3 * r + 1] +
                          p->base_dir[3 * r + 2] * p->base_dir[3 * r + 2]);
    if (!(nn > 0.0)) return bad("zero base_dir");
    int ax = -1;
    for (int k = 0; k < 3; ++k) {
      bd[3 * r + k] = p->base_dir[3 * r + k] / nn;
      if (std::fabs(std::fabs(bd[3 * r + k]) - 1.0) < 1e-15) ax = k;
    }
    if (p->guide_len > 0.0) {
      if (ax < 0) return bad("guide_len > 0 needs base_dir along a coordinate axis");
      gaxis[r] = ax;
    }
    double cx = bd[3 * r + 1] * bu[3 * r + 2] - bd[3 * r + 2] * bu[3 * r + 1];
    double cy = bd[3 * r + 2] * bu[3 * r] - bd[3 * r] * bu[3 * r + 2];
    double cz = bd[3 * r] * bu[3 * r + 1] - bd[3 * r + 1] * bu[3 * r];
    if (!(cx * cx + cy * cy + cz * cz > 1e-24)) return bad("base_up parallel to base_dir");
  }
  c->Ntot = c->h_off[c->B];
  const int64_t N = c->Ntot;
  const int B = c->B;
  const int cap = p->contact_capacity;
  Dev& d = c->d;
  d.B = B;
  d.Ntot = N;
  // robots
  int64_t* off_d; int32_t* robot_of; double *l0_d, *bp_d, *bd_d, *bu_d; int32_t* gax_d;
  ALLOC(off_d, B + 1); ALLOC(robot_of, N); ALLOC(l0_d, B); ALLOC(bp_d, 3 * B); ALLOC(bd_d, 3 * B);
  ALLOC(bu_d, 3 * B); ALLOC(gax_d, B);
  std::vector<int32_t> h_robot_of(N);
  for (int r = 0; r < B; ++r)
    for (int64_t g = c->h_off[r]; g < c->h_off[r + 1]; ++g) h_robot_of[g] = r;
  HIP_TRY(c, hipMemcpy(off_d, c->h_off.data(), (B + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(robot_of, h_robot_of.data(), N * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(l0_d, l0.data(), B * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(bp_d, bp.data(), 3 * B * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(bd_d, bd.data(), 3 * B * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(bu_d, bu.data(), 3 * B * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(gax_d, gaxis.data(), B * sizeof(int32_t), hipMemcpyHostToDevice));
  double* stag_d;
  ALLOC(stag_d, B);
  HIP_TRY(c, hipMemcpy(stag_d, stag.data(), B * sizeof(double), hipMemcpyHostToDevice));
  d.stag_r = stag_d;
  d.off = off_d; d.robot_of = robot_of; d.l0 = l0_d; d.base_pos = bp_d; d.base_dir = bd_d;
  d.base_up = bu_d; d.guide_axis = gax_d;
  {
    // robots by decreasing length: the step solve runs neighbours in this order side by side
    std::vector<int32_t> order(B);
    for (int r = 0; r < B; ++r) order[r] = r;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return c->h_nelem[a] > c->h_nelem[b]; });
    int32_t* order_d;
    ALLOC(order_d, B);
    HIP_TRY(c, hipMemcpy(order_d, order.data(), B * sizeof(int32_t), hipMemcpyHostToDevice));
    d.solve_order = order_d;
  }
  ALLOC(c->length_d, B);
  HIP_TRY(c, hipMemcpy(c->length_d, c->h_len.data(), B * sizeof(double), hipMemcpyHostToDevice));
  double *EA, *EI, *GJ;
  ALLOC(EA, N); ALLOC(EI, N); ALLOC(GJ, N);
  d.EA = EA; d.EI = EI; d.GJ = GJ;
  // cables
  double *cc, *cs;
  ALLOC(cc, p->n_cables); ALLOC(cs, p->n_cables);
  std::vector<double> hc(p->n_cables), hs(p->n_cables);
  for (int j = 0; j < p->n_cables; ++j) { hc[j] = std::cos(p->cable_angle[j]); hs[j] = std::sin(p->cable_angle[j]); }
  HIP_TRY(c, hipMemcpy(cc, hc.data(), p->n_cables * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(cs, hs.data(), p->n_cables * sizeof(double), hipMemcpyHostToDevice));
  d.n_cables = p->n_cables; d.cable_radius = p->cable_radius; d.cable_cos = cc; d.cable_sin = cs;
  // actuation buffers (max 8 values per robot)
  const int NV = 8;
  ALLOC(c->act_prev, NV * B); ALLOC(c->act_tgt, NV * B); ALLOC(c->act_cur, NV * B);
  ALLOC(c->dep_prev, B); ALLOC(c->dep_tgt, B); ALLOC(c->dep_cur, B);
  HIP_TRY(c, hipMemset(c->act_prev, 0, NV * B * sizeof(double)));
  HIP_TRY(c, hipMemset(c->act_tgt, 0, NV * B * sizeof(double)));
  HIP_TRY(c, hipMemset(c->act_cur, 0, NV * B * sizeof(double)));
  HIP_TRY(c, hipMemset(c->dep_prev, 0, B * sizeof(double)));
  HIP_TRY(c, hipMemset(c->dep_tgt, 0, B * sizeof(double)));
  HIP_TRY(c, hipMemset(c->dep_cur, 0, B * sizeof(double)));
  d.act_cur = c->act_cur; d.depth_cur = c->dep_cur; d.act_kind = 0; d.act_nv = p->n_cables;
  d.guide_len = p->guide_len;
  d.r_c = p->contact_radius; d.delta = p->contact_margin; d.beta0 = p->beta0;
  d.elements = p->contact_along_elements;
  d.newton_tol = p->newton_tol; d.stag_tol = p->stag_tol; d.max_newton = p->max_newton;
  d.cap = cap;
  d.mixed = (p->precision == FEM_MIXED) ? 1 : 0;
  // state and per-iteration buffers
  ALLOC(d.X, 7 * N); ALLOC(d.F, 6 * N); ALLOC(d.E1, 3 * N); ALLOC(d.E1f, 3 * N);
  double* kc = nullptr;
  ALLOC(kc, 6 * N);
  d.KC = kc;
  c->kc = kc;
  ALLOC(d.LD, 36 * N); ALLOC(d.LS, 36 * N);
  ALLOC(d.CC, N); ALLOC(d.CT, MAXC * N); ALLOC(d.CK, MAXC * N); ALLOC(d.CN, 3 * MAXC * N);
  ALLOC(d.CG, MAXC * N); ALLOC(d.CS, MAXC * N); ALLOC(d.CW, MAXC * N);
  HIP_TRY(c, hipMemset(d.CC, 0, N * sizeof(int32_t)));
  const int64_t BC = (int64_t)B * cap;
  ALLOC(d.ct_node, BC); ALLOC(d.ct_tri, BC); ALLOC(d.ct_kind, BC); ALLOC(d.ct_n, 3 * BC);
  ALLOC(d.ct_gap, BC); ALLOC(d.ct_y, BC); ALLOC(d.ct_s, BC); ALLOC(d.ct_warm, BC);
  ALLOC(d.cp_node, BC); ALLOC(d.cp_tri, BC); ALLOC(d.cp_kind, BC); ALLOC(d.cp_n, 3 * BC);
  ALLOC(d.cp_gap, BC); ALLOC(d.cp_y, BC); ALLOC(d.cp_s, BC);
  std::vector<int64_t> zoff(B);
  int64_t zt = 0;
  for (int r = 0; r < B; ++r) { zoff[r] = zt; zt += 6 * (int64_t)(c->h_nelem[r] + 1); }
  int64_t* zoff_d;
  ALLOC(zoff_d, B);
  HIP_TRY(c, hipMemcpy(zoff_d, zoff.data(), B * sizeof(int64_t), hipMemcpyHostToDevice));
  d.zoff = zoff_d;
  d.zp = ((int64_t)cap + 1 + 7) / 8 * 8;
  ALLOC(d.Y, 6 * d.zp * N);
  ALLOC(d.Z, zt);
  ALLOC(d.XM, (int64_t)B * SOLVE_THREADS * 6);
  ALLOC(d.W, (int64_t)B * cap * d.zp + (int64_t)B * lcp_ws_doubles(cap));
  ALLOC(d.q, BC);
  ALLOC(d.ac_idx, BC); ALLOC(d.ac_y, BC);
  ALLOC(d.st_nact, B); ALLOC(d.st_mx, B);
  ALLOC(d.wl, (int64_t)WL_SUB * B);
  ALLOC(d.wl_sub, (int64_t)B * ((cap + SOLVE_THREADS) / SOLVE_THREADS));
  ALLOC(d.wl_cnt, 8);
  HIP_TRY(c, hipMemset(d.wl_cnt, 0, 8 * sizeof(int32_t)));
  ALLOC(d.st_status, B); ALLOC(d.st_done, B); ALLOC(d.st_nc, B); ALLOC(d.st_ncp, B);
  ALLOC(d.st_limited, B); ALLOC(d.st_nlim, B); ALLOC(d.st_nswitch, B); ALLOC(d.st_iters, B); ALLOC(d.st_rhs, 5 * B);
  ALLOC(d.st_rn, B); ALLOC(d.st_rnprev, B); ALLOC(d.n_done, 1);
  ALLOC(d.st_step, B); ALLOC(d.st_it, B); ALLOC(d.st_fin, B);
  HIP_TRY(c, hipMemset(d.st_step, 0, B * sizeof(int32_t)));
  HIP_TRY(c, hipMemset(d.st_it, 0, B * sizeof(int32_t)));
  HIP_TRY(c, hipMemset(d.st_fin, 0, B * sizeof(int32_t)));
  d.act_prev = c->act_prev; d.act_tgt = c->act_tgt; d.dep_prev = c->dep_prev; d.dep_tgt = c->dep_tgt;
  d.sched_act = nullptr; d.sched_dep = nullptr;
  d.rec_tip = nullptr; d.rec_status = nullptr; d.rec_iters = nullptr;
  d.n_steps = 1;
  d.coll_lanes = 8;
  d.elem_block = 256;
  d.qp_admm = p->qp_solver == FEM_QP_ADMM ? 1 : 0;
  d.admm_rho = p->admm_rho > 0.0 ? p->admm_rho : 1.0;
  d.admm_eps = p->admm_eps > 0.0 ? p->admm_eps : 1e-11;
  d.admm_max_iter = p->admm_max_iter > 0 ? p->admm_max_iter : 20000;
  ALLOC(d.st_qpit, B);
  ALLOC(c->tune_save, B);
  HIP_TRY(c, hipMemset(d.st_qpit, 0, B * sizeof(int64_t)));
  HIP_TRY(c, hipMemset(d.st_status, 0, B * sizeof(int32_t)));
  HIP_TRY(c, hipMemset(d.st_done, 0, B * sizeof(int32_t)));
  HIP_TRY(c, hipMemset(d.st_nc, 0, B * sizeof(int32_t)));
  HIP_TRY(c, hipMemset(d.st_ncp, 0, B * sizeof(int32_t)));
  HIP_TRY(c, hipMemset(d.st_nlim, 0, B * sizeof(int32_t)));
  HIP_TRY(c, hipMemset(d.st_iters, 0, B * sizeof(int32_t)));
  HIP_TRY(c, hipMemset(d.st_rhs, 0, 5 * B * sizeof(int64_t)));
  HIP_TRY(c, hipMemset(d.st_rn, 0, B * sizeof(double)));
  ALLOC(c->steps_conv, B); ALLOC(c->steps_tot, B); ALLOC(c->iters_tot, B);
  d.steps_conv = c->steps_conv; d.steps_tot = c->steps_tot; d.iters_tot = c->iters_tot;
  HIP_TRY(c, hipMemset(c->steps_conv, 0, B * sizeof(int32_t)));
  HIP_TRY(c, hipMemset(c->steps_tot, 0, B * sizeof(int32_t)));
  HIP_TRY(c, hipMemset(c->iters_tot, 0, B * sizeof(int64_t)));
  // empty mesh until fem_set_lumen
  d.n_tris = 0;
  d.g_dim[0] = d.g_dim[1] = d.g_dim[2] = 0;
  d.g_h = 1.0;
  d.g_org[0] = d.g_org[1] = d.g_org[2] = 0.0;
  d.tv = nullptr; d.tsd = nullptr; d.tsf = nullptr; d.tqf = nullptr;
  d.cell_start = nullptr; d.cell_tris = nullptr; d.cell_sd = nullptr; d.cell_sf = nullptr;
  if (p->profile) {
    c->profile = true;
    HIP_TRY(c, hipEventCreate(&c->ev0));
    HIP_TRY(c, hipEventCreate(&c->ev1));
  }
  HIP_TRY(c, hipHostMalloc((void**)&c->h_done, sizeof(int32_t), hipHostMallocDefault));
  if (!c->stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking));
  HIP_TRY(c, hipStreamCreateWithFlags(&c->side_stream, hipStreamNonBlocking));
  for (hipEvent_t& e : c->fork_ev) HIP_TRY(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  hipLaunchKernelGGL(init_state_kernel, dim3(nblk(N, 256)), dim3(256), 0, c->stream, d, p->r_out,
                     p->r_in, p->E, p->nu, p->tip_len, p->shaft_E, p->shaft_A, p->shaft_I,
                     (const double*)c->length_d, c->kc);
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return FEM_OK;
}

// Sharp convex features of the wall (where a contact along an element is made): an edge shared
// by two triangles that each have the other's far vertex behind their plane (convex seen from
// the lumen) and whose unit normals have a dot product <= cos 10 deg; an edge of one triangle
// (a rim) or of more than two; a vertex on such an edge.  Per triangle: bits 0-2 the edges ab,
// ac, bc, bits 3-5 the vertices a, b, c.
static void sharp_features(const std::vector<double>& V, const std::vector<int32_t>& T,
                           const std::vector<double>& n, int64_t n_tris, int64_t n_verts,
                           std::vector<uint8_t>& out) {
  const double cos_fold = std::cos(10.0 * 3.14159265358979323846 / 180.0);
  const int ei[3][2] = {{0, 1}, {0, 2}, {1, 2}};
  std::vector<std::pair<uint64_t, int64_t>> edges;       // (key, 3 t + e)
  edges.reserve(3 * n_tris);
  for (int64_t t = 0; t < n_tris; ++t)
    for (int e = 0; e < 3; ++e) {
      const uint64_t u = (uint32_t)T[3 * t + ei[e][0]], v = (uint32_t)T[3 * t + ei[e][1]];
      edges.emplace_back((std::min(u, v) << 32) | std::max(u, v), 3 * t + e);
    }
  std::sort(edges.begin(), edges.end());
  out.assign(n_tris, 0);
  std::vector<uint8_t> vsharp(n_verts, 0);
  for (size_t i = 0; i < edges.size();) {
    size_t j = i;
    while (j < edges.size() && edges[j].first == edges[i].first) ++j;
    bool flag = true;
    if (j - i == 2) {
      const int64_t t = edges[i].second / 3, t2 = edges[i + 1].second / 3;
      const int64_t u = edges[i].first >> 32, v = edges[i].first & 0xffffffffull;
      auto far = [&](int64_t tt) {
        for (int k = 0; k < 3; ++k)
          if (T[3 * tt + k] != u && T[3 * tt + k] != v) return (int64_t)T[3 * tt + k];
        return (int64_t)T[3 * tt];
      };
      auto behind = [&](int64_t tt, int64_t w) {   // n_tt . (V_w - V_u) < 0
        double s = 0.0;
        for (int k = 0; k < 3; ++k) s += n[3 * tt + k] * (V[3 * w + k] - V[3 * u + k]);
        return s < 0.0;
      };
      double dn = 0.0;
      for (int k = 0; k < 3; ++k) dn += n[3 * t + k] * n[3 * t2 + k];
      flag = behind(t, far(t2)) && behind(t2, far(t)) && dn <= cos_fold;
    }
    for (size_t k = i; k < j; ++k)
      if (flag) out[edges[k].second / 3] |= (uint8_t)(1u << (edges[k].second % 3));
    if (flag) {
      vsharp[edges[i].first >> 32] = 1;
      vsharp[edges[i].first & 0xffffffffull] = 1;
    }
    i = j;
  }
  for (int64_t t = 0; t < n_tris; ++t)
    for (int k = 0; k < 3; ++k)
      if (vsharp[T[3 * t + k]]) out[t] |= (uint8_t)(1u << (3 + k));
}

fem_status fem_set_lumen(fem_ctx* c, const double* verts, int64_t n_verts, const int32_t* tris,
                         int64_t n_tris) {
  if (!c) return FEM_E_INVAL;
  if (n_tris < 0 || n_verts < 0 || (n_tris > 0 && (!verts || !tris || n_verts < 3)))
    return fail(c, FEM_E_INVAL, "bad mesh sizes or NULL arrays");
  if (n_tris > (int64_t)1 << 30) return fail(c, FEM_E_INVAL, "too many triangles");
  hipSetDevice(c->device);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (void* p : c->mesh_allocs) hipFree(p);
  c->mesh_allocs.clear();
  Dev& d = c->d;
  d.n_tris = 0;
  if (n_tris == 0) {
    c->lumen_set = true;
    return FEM_OK;
  }
  // host copies for validation and the grid
  std::vector<double> hv(3 * n_verts);
  std::vector<int32_t> ht(3 * n_tris);
  if (c->io_dev) {
    HIP_TRY(c, hipMemcpy(hv.data(), verts, hv.size() * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(ht.data(), tris, ht.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  } else {
    std::memcpy(hv.data(), verts, hv.size() * sizeof(double));
    std::memcpy(ht.data(), tris, ht.size() * sizeof(int32_t));
  }
  for (int64_t k = 0; k < 3 * n_tris; ++k)
    if (ht[k] < 0 || ht[k] >= n_verts) return fail(c, FEM_E_INVAL, "triangle vertex index out of range");
  for (int64_t t = 0; t < n_tris; ++t) {
    const double* a = &hv[3 * (int64_t)ht[3 * t]];
    const double* b = &hv[3 * (int64_t)ht[3 * t + 1]];
    const double* e = &hv[3 * (int64_t)ht[3 * t + 2]];
    double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, v[3] = {e[0] - a[0], e[1] - a[1], e[2] - a[2]};
    double n2 = std::pow(u[1] * v[2] - u[2] * v[1], 2) + std::pow(u[2] * v[0] - u[0] * v[2], 2) +
                std::pow(u[0] * v[1] - u[1] * v[0], 2);
    if (!(n2 > 0.0)) return fail(c, FEM_E_INVAL, "degenerate triangle " + std::to_string(t));
  }
  double *V_d, *tv;
  int32_t* T_d;
  double4* tsd;
  float4 *tsf, *tqf;
  auto A = [&](auto** ptr, size_t count) { return dalloc(c, ptr, count, c->mesh_allocs); };
  if (A(&V_d, 3 * n_verts) || A(&T_d, 3 * n_tris) || A(&tv, 12 * n_tris) ||
      A(&tsd, n_tris) || A(&tsf, n_tris) || A(&tqf, 4 * n_tris))
    return FEM_E_NOMEM;
  HIP_TRY(c, hipMemcpy(V_d, hv.data(), hv.size() * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(T_d, ht.data(), ht.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  launch_tri_setup(V_d, T_d, n_tris, tv, tsd, tsf, tqf, c->stream);
  HIP_TRY(c, hipGetLastError());
  // sharp convex features, where contacts along elements are made: per triangle bits 0-2 the
  // edges ab, ac, bc, bits 3-5 the vertices a, b, c
  {
    std::vector<double> nrm(3 * n_tris);
    for (int64_t t = 0; t < n_tris; ++t) {
      const double* a = &hv[3 * (int64_t)ht[3 * t]];
      const double* b = &hv[3 * (int64_t)ht[3 * t + 1]];
      const double* e = &hv[3 * (int64_t)ht[3 * t + 2]];
      const double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, v[3] = {e[0] - a[0], e[1] - a[1], e[2] - a[2]};
      const double x[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
      const double l = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
      for (int k = 0; k < 3; ++k) nrm[3 * t + k] = x[k] / l;
    }
    std::vector<uint8_t> hs;
    sharp_features(hv, ht, nrm, n_tris, n_verts, hs);
    uint8_t* ts_d;
    if (A(&ts_d, n_tris)) return FEM_E_NOMEM;
    HIP_TRY(c, hipMemcpy(ts_d, hs.data(), n_tris, hipMemcpyHostToDevice));
    d.tsharp = ts_d;
  }
  // uniform grid: every triangle in each cell its box grown by the band overlaps
  const double band = c->p.contact_radius + c->p.contact_margin;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t k = 0; k < n_verts; ++k)
    for (int j = 0; j < 3; ++j) { lo[j] = std::min(lo[j], hv[3 * k + j]); hi[j] = std::max(hi[j], hv[3 * k + j]); }
  double h = c->p.grid_cell > 0.0 ? c->p.grid_cell : band;
  int dim[3];
  for (;;) {
    int64_t cells = 1;
    for (int j = 0; j < 3; ++j) {
      dim[j] = (int)std::ceil((hi[j] - lo[j] + 2.0 * band) / h) + 1;
      cells *= dim[j];
    }
    if (cells <= (int64_t)64 << 20) break;
    h *= 1.25;
  }
  double org[3] = {lo[0] - band, lo[1] - band, lo[2] - band};
  const int64_t ncell = (int64_t)dim[0] * dim[1] * dim[2];
  std::vector<int32_t> cnt(ncell + 1, 0);
  auto cell_range = [&](int64_t t, int* c0, int* c1) {
    for (int j = 0; j < 3; ++j) {
      double mn = 1e300, mx = -1e300;
      for (int k = 0; k < 3; ++k) {
        double x = hv[3 * (int64_t)ht[3 * t + k] + j];
        mn = std::min(mn, x);
        mx = std::max(mx, x);
      }
      c0[j] = std::max(0, (int)std::floor((mn - band - org[j]) / h));
      c1[j] = std::min(dim[j] - 1, (int)std::floor((mx + band - org[j]) / h));
    }
  };
  int64_t total = 0;
  for (int64_t t = 0; t < n_tris; ++t) {
    int c0[3], c1[3];
    cell_range(t, c0, c1);
    for (int z = c0[2]; z <= c1[2]; ++z)
      for (int y = c0[1]; y <= c1[1]; ++y)
        for (int x = c0[0]; x <= c1[0]; ++x) { ++cnt[((int64_t)z * dim[1] + y) * dim[0] + x + 1]; ++total; }
  }
  if (total > ((int64_t)1 << 31) - 1) return fail(c, FEM_E_INVAL, "grid too large; raise grid_cell");
  for (int64_t k = 0; k < ncell; ++k) cnt[k + 1] += cnt[k];
  std::vector<int32_t> fillp(cnt.begin(), cnt.end() - 1), lst(std::max<int64_t>(total, 1));
  for (int64_t t = 0; t < n_tris; ++t) {
    int c0[3], c1[3];
    cell_range(t, c0, c1);
    for (int z = c0[2]; z <= c1[2]; ++z)
      for (int y = c0[1]; y <= c1[1]; ++y)
        for (int x = c0[0]; x <= c1[0]; ++x) lst[fillp[((int64_t)z * dim[1] + y) * dim[0] + x]++] = (int32_t)t;
  }
  int32_t *cs_d, *ct_d;
  double4* csd;
  float4* csf;
  if (A(&cs_d, ncell + 1) || A(&ct_d, lst.size()) || A(&csd, lst.size()) || A(&csf, lst.size()))
    return FEM_E_NOMEM;
  HIP_TRY(c, hipMemcpy(cs_d, cnt.data(), (ncell + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(ct_d, lst.data(), lst.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  // each cell entry carries its triangle's bounding spheres (contiguous reads in the cell walk)
  launch_cell_spheres(ct_d, (int64_t)lst.size(), tsd, tsf, csd, csf, c->stream);
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  d.n_tris = n_tris;
  d.tv = tv; d.tsd = tsd; d.tsf = tsf; d.tqf = tqf;
  d.g_h = h;
  for (int j = 0; j < 3; ++j) { d.g_org[j] = org[j]; d.g_dim[j] = dim[j]; }
  d.cell_start = cs_d; d.cell_tris = ct_d; d.cell_sd = csd; d.cell_sf = csf;
  c->lumen_set = true;
  return FEM_OK;
}

fem_status fem_set_actuation(fem_ctx* c, fem_act_kind kind, const double* values,
                             const double* insertion_depth) {
  if (!c) return FEM_E_INVAL;
  if (kind < FEM_ACT_CABLES || kind > FEM_ACT_CABLE_WRENCH || !values)
    return fail(c, FEM_E_INVAL, "bad actuation kind or NULL values");
  const int nv = (kind == FEM_ACT_CABLES || kind == FEM_ACT_CABLE_WRENCH) ? c->p.n_cables : 6;
  if (c->act_kind >= 0 && c->act_kind != (int)kind)
    return fail(c, FEM_E_INVAL, "actuation kind cannot change");
  hipSetDevice(c->device);
  c->act_kind = kind;
  c->act_nv = nv;
  c->d.act_kind = kind;
  c->d.act_nv = nv;
  fem_status s = copy_in(c, c->act_tgt, values, (size_t)c->B * nv * sizeof(double));
  if (s != FEM_OK) return s;
  if (insertion_depth) {
    s = copy_in(c, c->dep_tgt, insertion_depth, (size_t)c->B * sizeof(double));
    if (s != FEM_OK) return s;
  } else {
    HIP_TRY(c, hipMemsetAsync(c->dep_tgt, 0, c->B * sizeof(double), c->stream));
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->act_set = true;
  return FEM_OK;
}

fem_status fem_get_state(const fem_ctx* cc, double* node_state) {
  fem_ctx* c = const_cast<fem_ctx*>(cc);
  if (!c || !node_state) return FEM_E_INVAL;
  hipSetDevice(c->device);
  double* tmp = c->d.F;  // scratch of 6N is too small for 7N: use LD (36N)
  tmp = c->d.LD;
  hipLaunchKernelGGL(soa_to_aos, dim3(nblk(c->Ntot, 256)), dim3(256), 0, c->stream, c->d.X, tmp,
                     c->Ntot, 7);
  HIP_TRY(c, hipGetLastError());
  return copy_out(c, node_state, tmp, (size_t)c->Ntot * 7 * sizeof(double));
}

fem_status fem_set_state(fem_ctx* c, const double* node_state) {
  if (!c || !node_state) return FEM_E_INVAL;
  hipSetDevice(c->device);
  double* tmp = c->d.LD;
  fem_status s = copy_in(c, tmp, node_state, (size_t)c->Ntot * 7 * sizeof(double));
  if (s != FEM_OK) return s;
  hipLaunchKernelGGL(aos_to_soa, dim3(nblk(c->Ntot, 256)), dim3(256), 0, c->stream, tmp, c->d.X,
                     c->Ntot, 7);
  hipLaunchKernelGGL(renorm_kernel, dim3(nblk(c->Ntot, 256)), dim3(256), 0, c->stream, c->d);
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipMemsetAsync(c->steps_conv, 0, c->B * sizeof(int32_t), c->stream));
  HIP_TRY(c, hipMemsetAsync(c->steps_tot, 0, c->B * sizeof(int32_t), c->stream));
  HIP_TRY(c, hipMemsetAsync(c->iters_tot, 0, c->B * sizeof(int64_t), c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d.st_rhs, 0, 5 * c->B * sizeof(int64_t), c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d.st_qpit, 0, c->B * sizeof(int64_t), c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->solved = false;
  return FEM_OK;
}

// after the load steps of a call: the target is reached (the start of the next ramp, also
// for zero load steps); per-robot records and the state are written out
static fem_status solve_epilogue(fem_ctx* c, double* node_state, fem_solve_info* info) {
  const int B = c->B;
  Dev& d = c->d;
  HIP_TRY(c, hipMemcpyAsync(c->act_prev, c->act_tgt, (size_t)B * 8 * sizeof(double),
                            hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->dep_prev, c->dep_tgt, (size_t)B * sizeof(double),
                            hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  bool any_fail = false;
  std::vector<int32_t> st(B);
  HIP_TRY(c, hipMemcpy(st.data(), d.st_status, B * sizeof(int32_t), hipMemcpyDeviceToHost));
  for (int r = 0; r < B; ++r) any_fail |= (st[r] != 0);
  if (info) {
    std::vector<int32_t> it(B), nc(B), nl(B), sc(B), stt(B);
    std::vector<double> rn(B);
    std::vector<int64_t> itt(B);
    HIP_TRY(c, hipMemcpy(it.data(), d.st_iters, B * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(nc.data(), d.st_ncp, B * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(nl.data(), d.st_nlim, B * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(rn.data(), d.st_rn, B * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(sc.data(), c->steps_conv, B * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(stt.data(), c->steps_tot, B * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(itt.data(), c->iters_tot, B * sizeof(int64_t), hipMemcpyDeviceToHost));
    std::vector<int64_t> rhs(5 * B), qpit(B);
    HIP_TRY(c, hipMemcpy(rhs.data(), d.st_rhs, 5 * B * sizeof(int64_t), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(qpit.data(), d.st_qpit, B * sizeof(int64_t), hipMemcpyDeviceToHost));
    std::vector<fem_solve_info> hi(B);
    for (int r = 0; r < B; ++r) {
      hi[r].status = st[r]; hi[r].iters = it[r]; hi[r].n_contacts = nc[r]; hi[r].n_limited = nl[r];
      hi[r].res_norm = rn[r]; hi[r].steps_converged = sc[r]; hi[r].steps_total = stt[r];
      hi[r].iters_total = itt[r];
      hi[r].rhs_total = rhs[5 * r];
      hi[r].rhs_fused = rhs[5 * r + 1];
      hi[r].sweep_passes = rhs[5 * r + 2];
      hi[r].qp_iters_total = qpit[r];
      hi[r].products_total = rhs[5 * r + 3];
      hi[r].contact_steps_total = rhs[5 * r + 4];
    }
    if (c->io_dev) {
      HIP_TRY(c, hipMemcpy(info, hi.data(), B * sizeof(fem_solve_info), hipMemcpyHostToDevice));
    } else {
      std::memcpy(info, hi.data(), B * sizeof(fem_solve_info));
    }
  }
  if (node_state) {
    fem_status s = fem_get_state(c, node_state);
    if (s != FEM_OK) return s;
  }
  return any_fail ? FEM_E_NOCONV : FEM_OK;
}

fem_status fem_solve(fem_ctx* c, int32_t n_load_steps, double* node_state, fem_solve_info* info) {
  if (!c) return FEM_E_INVAL;
  if (n_load_steps < 0) return fail(c, FEM_E_INVAL, "n_load_steps < 0");
  if (!c->lumen_set) return fail(c, FEM_E_STATE, "fem_set_lumen was not called");
  if (!c->act_set) return fail(c, FEM_E_STATE, "fem_set_actuation was not called");
  hipSetDevice(c->device);
  Dev& d = c->d;
  d.sched_act = nullptr; d.sched_dep = nullptr;
  d.rec_tip = nullptr; d.rec_status = nullptr; d.rec_iters = nullptr;
  if (n_load_steps > 0) {
    fem_status s = run_load_steps(c, n_load_steps);
    if (s != FEM_OK) return s;
    c->solved = true;
  }
  return solve_epilogue(c, node_state, info);
}

fem_status fem_solve_schedule(fem_ctx* c, fem_act_kind kind, int32_t n_load_steps,
                              const double* values, const double* insertion_depth,
                              double* node_state, fem_solve_info* info, double* rec_tip,
                              int32_t* rec_status, int32_t* rec_iters) {
  if (!c) return FEM_E_INVAL;
  if (n_load_steps < 1) return fail(c, FEM_E_INVAL, "n_load_steps < 1");
  if (kind < FEM_ACT_CABLES || kind > FEM_ACT_CABLE_WRENCH || !values)
    return fail(c, FEM_E_INVAL, "bad actuation kind or NULL values");
  if (c->act_kind >= 0 && c->act_kind != (int)kind)
    return fail(c, FEM_E_INVAL, "actuation kind cannot change");
  if (!c->lumen_set) return fail(c, FEM_E_STATE, "fem_set_lumen was not called");
  hipSetDevice(c->device);
  const int B = c->B;
  const int nv = (kind == FEM_ACT_CABLES || kind == FEM_ACT_CABLE_WRENCH) ? c->p.n_cables : 6;
  const int64_t nsb = (int64_t)n_load_steps * B;
  Dev& d = c->d;
  c->act_kind = kind;
  c->act_nv = nv;
  d.act_kind = kind;
  d.act_nv = nv;
  // the schedule in device memory
  const double* sa = values;
  const double* sd = insertion_depth;
  if (!c->io_dev) {
    const int64_t need = nsb * (nv + 1);
    if (need > c->sched_cap) {
      if (c->sched_buf) (void)hipFree(c->sched_buf);
      c->sched_buf = nullptr;
      c->sched_cap = 0;
      if (hipMalloc(&c->sched_buf, need * sizeof(double)) != hipSuccess)
        return fail(c, FEM_E_NOMEM, "hipMalloc of the schedule failed");
      c->sched_cap = need;
    }
    HIP_TRY(c, hipMemcpy(c->sched_buf, values, nsb * nv * sizeof(double), hipMemcpyHostToDevice));
    sa = c->sched_buf;
    if (insertion_depth) {
      HIP_TRY(c, hipMemcpy(c->sched_buf + nsb * nv, insertion_depth, nsb * sizeof(double),
                           hipMemcpyHostToDevice));
      sd = c->sched_buf + nsb * nv;
    }
  } else {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  // per-step records in device memory: tips (doubles), then status and iterations (int32)
  double* rt = rec_tip;
  int32_t* rs = rec_status;
  int32_t* ri = rec_iters;
  if (!c->io_dev && (rec_tip || rec_status || rec_iters)) {
    const int64_t need = nsb * 4;
    if (need > c->rec_cap) {
      if (c->rec_buf) (void)hipFree(c->rec_buf);
      c->rec_buf = nullptr;
      c->rec_cap = 0;
      if (hipMalloc(&c->rec_buf, need * sizeof(double)) != hipSuccess)
        return fail(c, FEM_E_NOMEM, "hipMalloc of the per-step records failed");
      c->rec_cap = need;
    }
    rt = rec_tip ? c->rec_buf : nullptr;
    rs = rec_status ? (int32_t*)(c->rec_buf + 3 * nsb) : nullptr;
    ri = rec_iters ? (int32_t*)(c->rec_buf + 3 * nsb) + nsb : nullptr;
  }
  // without depths the depth stays where the previous call left it
  if (!sd)
    HIP_TRY(c, hipMemcpy(c->dep_tgt, c->dep_prev, (size_t)B * sizeof(double), hipMemcpyDeviceToDevice));
  d.sched_act = sa; d.sched_dep = sd;
  d.rec_tip = rt; d.rec_status = rs; d.rec_iters = ri;
  c->act_set = true;
  fem_status s = run_load_steps(c, n_load_steps);
  d.sched_act = nullptr; d.sched_dep = nullptr;
  d.rec_tip = nullptr; d.rec_status = nullptr; d.rec_iters = nullptr;
  if (s != FEM_OK) return s;
  c->solved = true;
  // the last step's values are the target reached (the start of a later ramp)
  HIP_TRY(c, hipMemcpy(c->act_tgt, sa + (nsb - B) * nv, (size_t)B * nv * sizeof(double),
                       hipMemcpyDeviceToDevice));
  if (sd)
    HIP_TRY(c, hipMemcpy(c->dep_tgt, sd + (nsb - B), (size_t)B * sizeof(double), hipMemcpyDeviceToDevice));
  if (!c->io_dev) {
    if (rec_tip) HIP_TRY(c, hipMemcpy(rec_tip, rt, nsb * 3 * sizeof(double), hipMemcpyDeviceToHost));
    if (rec_status) HIP_TRY(c, hipMemcpy(rec_status, rs, nsb * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (rec_iters) HIP_TRY(c, hipMemcpy(rec_iters, ri, nsb * sizeof(int32_t), hipMemcpyDeviceToHost));
  }
  return solve_epilogue(c, node_state, info);
}

fem_status fem_grad(fem_ctx* c, const int32_t* sensor_nodes, int32_t n_sensors,
                    const double* dL_dp, double* dL_du) {
  if (!c) return FEM_E_INVAL;
  if (!sensor_nodes || !dL_dp || !dL_du || n_sensors < 1)
    return fail(c, FEM_E_INVAL, "fem_grad: NULL pointer or n_sensors < 1");
  int64_t min_nodes = INT64_MAX;
  for (int r = 0; r < c->B; ++r) min_nodes = std::min<int64_t>(min_nodes, c->h_off[r + 1] - c->h_off[r]);
  for (int s = 0; s < n_sensors; ++s) {
    const int64_t i = sensor_nodes[s];
    if (i >= min_nodes || i < -min_nodes)
      return fail(c, FEM_E_INVAL, "fem_grad: sensor node index outside a robot");
  }
  if (!c->solved || !c->act_set || !c->lumen_set)
    return fail(c, FEM_E_STATE, "fem_grad: no load step solved since creation or fem_set_state");
  hipSetDevice(c->device);
  const int B = c->B;
  const int64_t N = c->Ntot;
  Dev& d = c->d;
  if (!c->aJL) {
    ALLOC(c->aJL, N * 36); ALLOC(c->aJD, N * 36); ALLOC(c->aJU, N * 36);
    ALLOC(c->aQB, N * 9); ALLOC(c->aKF, N); ALLOC(c->aGP, N * 6);
    ALLOC(c->aout, (int64_t)B * 8); ALLOC(c->astat, B);
  }
  if (n_sensors > c->a_ns_cap) {
    ALLOC(c->asens, n_sensors);
    ALLOC(c->adLdp, (int64_t)B * n_sensors * 3);
    c->a_ns_cap = n_sensors;
  }
  HIP_TRY(c, hipMemcpyAsync(c->asens, sensor_nodes, n_sensors * sizeof(int32_t), hipMemcpyHostToDevice,
                            c->stream));
  fem_status st = copy_in(c, c->adLdp, dL_dp, (size_t)B * n_sensors * 3 * sizeof(double));
  if (st != FEM_OK) return st;
  launch_adjoint(d, c->asens, n_sensors, c->adLdp, c->aJL, c->aJD, c->aJU, c->aQB, c->aKF, c->aGP,
                 c->aout, c->astat, c->stream);
  HIP_TRY(c, hipGetLastError());
  st = copy_out(c, dL_du, c->aout, (size_t)B * c->act_nv * sizeof(double));
  if (st != FEM_OK) return st;
  std::vector<int32_t> rs(B);
  HIP_TRY(c, hipMemcpy(rs.data(), c->astat, B * sizeof(int32_t), hipMemcpyDeviceToHost));
  int n_bad = 0;
  for (int r = 0; r < B; ++r) n_bad += (rs[r] != 0);
  if (n_bad) return fail(c, FEM_E_NOCONV, "fem_grad: " + std::to_string(n_bad) +
                                              " robot(s) not converged, with a singular adjoint system or"
                                              " with an active contact along an element");
  return FEM_OK;
}

fem_status fem_profile(fem_ctx* c, int32_t kernel, double* total_ms, int64_t* launches,
                       int32_t reset) {
  if (!c) return FEM_E_INVAL;
  if (kernel < 0 || kernel > 6) return fail(c, FEM_E_INVAL, "kernel class must be 0..6");
  if (!c->profile) return fail(c, FEM_E_STATE, "context was created without profile = 1");
  if (total_ms) *total_ms = c->prof_ms[kernel];
  if (launches) *launches = c->prof_n[kernel];
  if (reset) {
    c->prof_ms[kernel] = 0.0;
    c->prof_n[kernel] = 0;
  }
  return FEM_OK;
}

fem_status fem_eval(fem_ctx* c, double* F, double* KD, double* KS) {
  if (!c) return FEM_E_INVAL;
  if (!c->lumen_set) return fail(c, FEM_E_STATE, "fem_set_lumen was not called");
  if (!c->act_set) return fail(c, FEM_E_STATE, "fem_set_actuation was not called");
  hipSetDevice(c->device);
  Dev& d = c->d;
  hipLaunchKernelGGL(set_load_kernel, dim3(nblk(c->B, 256)), dim3(256), 0, c->stream, d,
                     (const double*)c->act_prev, (const double*)c->act_tgt, c->act_cur,
                     (const double*)c->dep_prev, (const double*)c->dep_tgt, c->dep_cur, 1, 1);
  launch_elem(d, c->stream);
  launch_collide(d, c->stream);
  launch_gather(d, c->stream);
  HIP_TRY(c, hipGetLastError());
  if (F) {
    hipLaunchKernelGGL(soa_to_aos, dim3(nblk(c->Ntot, 256)), dim3(256), 0, c->stream, d.F, d.LS,
                       c->Ntot, 6);
    HIP_TRY(c, hipGetLastError());
    fem_status s = copy_out(c, F, d.LS, (size_t)c->Ntot * 6 * sizeof(double));
    if (s != FEM_OK) return s;
  }
  if (KD || KS) {
    hipLaunchKernelGGL(assemble_kernel, dim3(nblk(c->Ntot, 256)), dim3(256), 0, c->stream, d, d.LD,
                       d.LS);
    HIP_TRY(c, hipGetLastError());
    if (KD) {
      fem_status s = copy_out(c, KD, d.LD, (size_t)c->Ntot * 36 * sizeof(double));
      if (s != FEM_OK) return s;
    }
    if (KS) {
      fem_status s = copy_out(c, KS, d.LS, (size_t)c->Ntot * 36 * sizeof(double));
      if (s != FEM_OK) return s;
    }
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return FEM_OK;
}

fem_status fem_contacts(const fem_ctx* cc, int32_t robot, fem_contact* out, int32_t capacity,
                        int32_t* n_out) {
  fem_ctx* c = const_cast<fem_ctx*>(cc);
  if (!c || !n_out || capacity < 0 || (capacity > 0 && !out)) return FEM_E_INVAL;
  if (robot < -1 || robot >= c->B) return fail(c, FEM_E_INVAL, "robot index out of range");
  hipSetDevice(c->device);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int B = c->B, cap = c->p.contact_capacity;
  const Dev& d = c->d;
  std::vector<int32_t> ncp(B);
  HIP_TRY(c, hipMemcpy(ncp.data(), d.st_ncp, B * sizeof(int32_t), hipMemcpyDeviceToHost));
  const int r0 = robot < 0 ? 0 : robot, r1 = robot < 0 ? B : robot + 1;
  int64_t total = 0;
  for (int r = r0; r < r1; ++r) total += ncp[r];
  *n_out = (int32_t)std::min<int64_t>(total, INT32_MAX);
  std::vector<fem_contact> h;
  h.reserve(std::min<int64_t>(total, capacity));
  std::vector<int32_t> nd(cap), tr(cap), kd(cap);
  std::vector<double> nn(3 * cap), gp(cap), yy(cap), ss(cap);
  for (int r = r0; r < r1 && (int64_t)h.size() < capacity; ++r) {
    const int n = ncp[r];
    if (n == 0) continue;
    const int64_t cb = (int64_t)r * cap;
    HIP_TRY(c, hipMemcpy(nd.data(), d.cp_node + cb, n * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(tr.data(), d.cp_tri + cb, n * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(kd.data(), d.cp_kind + cb, n * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(nn.data(), d.cp_n + 3 * cb, 3 * n * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(gp.data(), d.cp_gap + cb, n * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(yy.data(), d.cp_y + cb, n * sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(ss.data(), d.cp_s + cb, n * sizeof(double), hipMemcpyDeviceToHost));
    for (int k = 0; k < n && (int64_t)h.size() < capacity; ++k) {
      fem_contact ct;
      ct.robot = r; ct.node = nd[k]; ct.tri = tr[k]; ct.kind = kd[k];
      ct.n[0] = nn[3 * k]; ct.n[1] = nn[3 * k + 1]; ct.n[2] = nn[3 * k + 2];
      ct.gap = gp[k]; ct.force = yy[k]; ct.s = ss[k];
      h.push_back(ct);
    }
  }
  if (!h.empty()) {
    if (c->io_dev) {
      HIP_TRY(c, hipMemcpy(out, h.data(), h.size() * sizeof(fem_contact), hipMemcpyHostToDevice));
    } else {
      std::memcpy(out, h.data(), h.size() * sizeof(fem_contact));
    }
  }
  return FEM_OK;
}

fem_status fem_lcp(const double* W, const double* q, int32_t m, double* y, int32_t* path) {
  if (!W || !q || !y || !path || m < 1 || m > 1024) return FEM_E_INVAL;
  const int64_t nw = (int64_t)m * m;
  double* dW = nullptr;     // W, then q, y, scratch (m*m + 3m) in one allocation
  int* dcode = nullptr;
  fem_status st = FEM_OK;
  if (hipMalloc(&dW, (2 * nw + 5 * (int64_t)m) * sizeof(double)) != hipSuccess) return FEM_E_NOMEM;
  if (hipMalloc(&dcode, sizeof(int)) != hipSuccess) {
    (void)hipFree(dW);
    return FEM_E_NOMEM;
  }
  double* dq = dW + nw;
  double* dy = dq + m;
  double* dscr = dy + m;
  int code = -1;
  if (hipMemcpy(dW, W, nw * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dq, q, m * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    st = FEM_E_HIP;
  } else {
    launch_lcp_check(dW, dq, m, dy, dscr, dcode, nullptr);
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(&code, dcode, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) {
      st = FEM_E_HIP;
    } else if (code < 0) {
      st = FEM_E_NOCONV;
    } else if (hipMemcpy(y, dy, m * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
      st = FEM_E_HIP;
    } else {
      *path = code;
    }
  }
  (void)hipFree(dcode);
  (void)hipFree(dW);
  return st;
}

}  // extern "C"

// ------------------------------------------------------------------ allocation-free LCP
// Device workspace of fem_lcp_noalloc: the factor workspace of the HBM-factor routine for up
// to FEM_LCP_NOALLOC_MAX_M constraints, followed by one slot for the routine's result code.
// Each GPU holds its own copy until the process ends; in host code the array's name is not a
// device address, so its address is taken once per device with hipGetSymbolAddress.
namespace {
constexpr int64_t kNoallocWs = (int64_t)FEM_LCP_NOALLOC_MAX_M * (FEM_LCP_NOALLOC_MAX_M + 1) / 2 +
                               3 * (int64_t)FEM_LCP_NOALLOC_MAX_M;
static_assert(kNoallocWs >= 1, "workspace");
__device__ __align__(256) double scratch[kNoallocWs + 1];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

extern "C" {

fem_status fem_lcp_noalloc(const double* W, const double* q, int32_t m, double* y, int32_t* path,
                           void* hip_stream) {
  if (!W || !q || !y || !path || m < 1 || m > FEM_LCP_NOALLOC_MAX_M) return FEM_E_INVAL;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return FEM_E_HIP;
  double* ws = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void* a = nullptr;
      if (hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)) != hipSuccess || !a) return FEM_E_HIP;
      g_scratch_ptr[dev] = static_cast<double*>(a);
    }
    ws = g_scratch_ptr[dev];
  }
  hipStream_t s = (hipStream_t)hip_stream;
  int* dcode = reinterpret_cast<int*>(ws + kNoallocWs);
  // the routines only read W (the dense source builds no columns)
  launch_lcp_check(const_cast<double*>(W), q, m, y, ws, dcode, s);
  if (hipGetLastError() != hipSuccess) return FEM_E_HIP;
  int code = -1;
  if (hipMemcpyAsync(&code, dcode, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return FEM_E_HIP;
  if (code < 0) return FEM_E_NOCONV;
  *path = code;
  return FEM_OK;
}

}  // extern "C"
