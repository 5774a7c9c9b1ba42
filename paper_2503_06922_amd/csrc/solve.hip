// Per-robot Newton step: contact gather, convergence test, block-tridiagonal
// Cholesky of the QP tangent, multi-right-hand-side solves, contact-space Schur
// complement, exact contact forces by an active-set method, step-size limit and
// state update.  One wavefront (64 lanes) per robot.  Kernels with a block per robot take
// the robots in order of decreasing length (the longest start first, so that the short
// ones fill in behind them).
//
// Linear step (eq. 20-23): with the base node prescribed (clamp + insertion,
// eq. 14-15) and the lateral DOFs of guided nodes prescribed on the guide axis,
//     K dx = -r + A^T y,   0 <= y  _|_  g + A dx >= 0,
// where A has one row n_c^T on the translations of each contact node (along an element:
// (1 - s) n_c^T on its base-side node and s n_c^T on the next).  With
// K = L L^T (6x6 blocks, serial over nodes), dx_free = -K^-1 r, Z = K^-1 A^T,
// W = A Z (SPD) and q = g + A dx_free, the contact forces solve LCP(q, W); the
// primal active-set method used here (Lawson-Hanson style, with a dense
// Cholesky of the active block) terminates finitely for SPD W.  Only the values of
// dx_free and Z at the contact nodes are needed for W and q: the substitution keeps the
// products n_i . (column)(node of i) and never stores whole columns.  Then
// dx = K^-1 (-r + A^T y) = dx_free + Z y by one more solve, and if max_i |dp_i| > beta the
// step and y are scaled by beta / max_i |dp_i| (eq. 25-27), beta = beta0 halved every 10
// contact-set changes within the load step (down to beta0/64).
//
// Convergence (checked at the start of the next iteration, after the state
// update, element update and detection): residual F - A_prev^T y_prev over the
// free DOFs (guided lateral DOFs excluded) below newton_tol, or below stag_tol
// and no longer halving; the last step unlimited; the detected contact set equal
// to the solved one; and no gap below -1e-9 m.  The stagnation level is stag_tol
// raised to ten times the rounding floor eps * max(EA)/l0 * (1 m) * sqrt(DOFs).
#include "fem_device.h"

namespace accfem {

constexpr int NT = SOLVE_THREADS;
constexpr int CH = 16;                     // nodes per staged chunk
constexpr int PF = (CH * 36 + NT - 1) / NT;  // prefetch registers per lane and array
constexpr int CHF = 32;                    // nodes per staged chunk of the factorisation sweep
constexpr int CHS = 6;                     // chunk of the substitution sweeps (register budget)
constexpr int PFS = ((CHS + 1) * 36 + NT - 1) / NT;

// Forward values are stored at checkpoint nodes only: the base side's sweep (ascending f)
// keeps the last node of every CHS-aligned chunk, the tip side's (descending f) the first, so
// that a backward sweep recomputes a chunk's forward values from the checkpoint before it
// with the factor blocks it stages anyway.
__device__ __forceinline__ bool checkpoint_node(bool tip_side, int64_t f) {
  return tip_side ? (f % CHS) == 0 : (f % CHS) == CHS - 1;
}

__device__ __forceinline__ double warp_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double warp_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double warp_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
// v of lane l (l the same on every lane): two scalar lane reads instead of a shuffle through LDS
__device__ __forceinline__ double lane_read(double v, int l) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ int warp_sum_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Nodes 1..last of robot r are inside the insertion guide at this load step
// (reference arc length i*l0 + depth < guide_len, evaluated without contraction so
// the decision matches an unfused multiply-add); their lateral DOFs are prescribed.
struct Guide {
  int ax;        // guide axis (coordinate index), -1 if no guide
  int64_t last;  // last guided node index, 0 if none
  __device__ __forceinline__ bool dof(int64_t i, int k) const {
    return ax >= 0 && i >= 1 && i <= last && k < 3 && k != ax;
  }
};

__device__ Guide make_guide(const Dev& d, int r, int64_t n) {
  Guide G;
  G.ax = d.guide_axis[r];
  int64_t last = 0;
  if (G.ax >= 0) {
    const double l0 = d.l0[r], dep = d.depth_cur[r];
    for (int64_t i = 1 + threadIdx.x % SOLVE_THREADS; i < n; i += SOLVE_THREADS)
      if (__dadd_rn(__dmul_rn((double)i, l0), dep) < d.guide_len) last = max(last, i);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) last = max(last, (int64_t)__shfl_xor((long long)last, o));
  }
  G.last = last;
  return G;
}

// compact the per-node detection output of robot r into its contact list
__device__ void gather_contacts(const Dev& d, int r, int* nc_out, bool* overflow) {
  const int lane = threadIdx.x;
  const int64_t o = d.off[r], n = d.off[r + 1] - o;
  const int64_t N = d.Ntot;
  const int64_t chunk = (n + NT - 1) / NT;
  const int64_t i0 = min(n, (int64_t)lane * chunk), i1 = min(n, i0 + chunk);
  int cnt = 0, ovf = 0;
  for (int64_t i = i0; i < i1; ++i) {
    int c = d.CC[o + i];
    if (c > MAXC) { ovf = 1; c = MAXC; }
    cnt += c;
  }
  // exclusive scan over the wavefront
  int incl = cnt;
#pragma unroll
  for (int s = 1; s < 64; s <<= 1) {
    int v = __shfl_up(incl, s);
    if (lane >= s) incl += v;
  }
  const int total = __shfl(incl, 63);
  int pos = incl - cnt;
  ovf = warp_sum_i(ovf);
  const int cap = d.cap;
  if (total <= cap && ovf == 0) {
    const int64_t base = (int64_t)r * cap;
    for (int64_t i = i0; i < i1; ++i) {
      const int64_t g = o + i;
      const int c = d.CC[g];
      for (int s = 0; s < c; ++s, ++pos) {
        d.ct_node[base + pos] = (int32_t)i;
        d.ct_tri[base + pos] = d.CT[s * N + g];
        d.ct_kind[base + pos] = d.CK[s * N + g];
        d.ct_warm[base + pos] = d.CW[s * N + g];
        d.ct_gap[base + pos] = d.CG[s * N + g];
        d.ct_s[base + pos] = d.CS[s * N + g];
        d.ct_n[3 * (base + pos) + 0] = d.CN[(3 * s + 0) * N + g];
        d.ct_n[3 * (base + pos) + 1] = d.CN[(3 * s + 1) * N + g];
        d.ct_n[3 * (base + pos) + 2] = d.CN[(3 * s + 2) * N + g];
      }
    }
  }
  *nc_out = total;
  *overflow = (total > cap) || (ovf != 0);
}

__device__ __forceinline__ void finish(const Dev& d, int r, int status, int iters, double rn) {
  if (threadIdx.x == 0) {
    d.st_status[r] = status;
    d.st_done[r] = 1;
    d.st_iters[r] = iters;
    d.st_rn[r] = rn;
  }
}

// phase 1: contact gather, convergence test, right-hand sides (col 0 = -r, contact columns)
__global__ void __launch_bounds__(NT) check_rhs_kernel(Dev d) {
  const int r = d.solve_order[blockIdx.x];   // longest robots first
  const int lane = threadIdx.x;
  if (d.st_done[r]) return;
  const int it = d.st_it[r];
  const int64_t o = d.off[r], n = d.off[r + 1] - o;
  const int64_t N = d.Ntot;
  const int64_t nf = n - 1;            // free nodes 1..n-1 -> f = 0..nf-1
  const int cap = d.cap;
  const int64_t cb = (int64_t)r * cap;
  const Guide G = make_guide(d, r, n);

  int nc;
  bool ovf;
  gather_contacts(d, r, &nc, &ovf);
  if (ovf) {
    if (lane == 0) d.st_nc[r] = nc;
    finish(d, r, 4, it, d.st_rn[r]);
    return;
  }
  __syncthreads();
  if (lane == 0) d.st_nc[r] = nc;

  // ---------------------------------------------------------------- convergence test
  if (it > 0) {
    const int ncp = d.st_ncp[r];
    int diff = (nc != ncp) ? 1 : 0;
    if (!diff) {
      for (int c = lane; c < nc; c += NT)
        diff |= (d.ct_node[cb + c] != d.cp_node[cb + c]) | (d.ct_tri[cb + c] != d.cp_tri[cb + c]) |
                (d.ct_kind[cb + c] != d.cp_kind[cb + c]);
      diff = warp_sum_i(diff);
    }
    double gmin = 1e300;
    for (int c = lane; c < nc; c += NT) gmin = fmin(gmin, d.ct_gap[cb + c]);
    gmin = warp_min(gmin);
    // residual over free nodes with the previous contact forces
    const int64_t chunk = (nf + NT - 1) / NT;
    const int64_t f0 = min(nf, (int64_t)lane * chunk), f1 = min(nf, f0 + chunk);
    double ss = 0.0;
    // contacts of node i (weight 1 - s) and contacts along the element i-1 -> i (weight s)
    int cp = 0;
    while (cp < ncp && d.cp_node[cb + cp] < f0) ++cp;
    for (int64_t f = f0; f < f1; ++f) {
      const int64_t i = f + 1, g = o + i;
      double rv[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) rv[k] = d.F[k * N + g];
      for (int c = cp; c < ncp && d.cp_node[cb + c] <= i; ++c) {
        const double sv = d.cp_s[cb + c];
        const double y = d.cp_y[cb + c] * (d.cp_node[cb + c] == i ? 1.0 - sv : sv);
        rv[0] -= y * d.cp_n[3 * (cb + c) + 0];
        rv[1] -= y * d.cp_n[3 * (cb + c) + 1];
        rv[2] -= y * d.cp_n[3 * (cb + c) + 2];
      }
      while (cp < ncp && d.cp_node[cb + cp] < i) ++cp;     // node i's contacts start node i+1's
#pragma unroll
      for (int k = 0; k < 6; ++k)
        if (!G.dof(i, k)) ss += rv[k] * rv[k];
    }
    ss = warp_sum(ss);
    const double rn = sqrt(ss);
    const double rn_prev = d.st_rnprev[r];
    const bool same = (diff == 0);
    // mixed precision: a residual of FP32 element forces never decides convergence
    const bool fp32_forces = d.mixed && d.st_rn[r] > F32_RESIDUAL;
    const bool conv = same && !d.st_limited[r] && gmin >= -1e-9 && !fp32_forces &&
                      (rn <= d.newton_tol || (rn <= d.stag_r[r] && rn > 0.5 * rn_prev));
    __syncthreads();
    if (lane == 0) {
      d.st_nswitch[r] += same ? 0 : 1;
      d.st_rnprev[r] = rn;
      d.st_rn[r] = rn;
    }
    if (conv) {
      // report the solved contacts with the gaps of the final state
      for (int c = lane; c < nc; c += NT) d.cp_gap[cb + c] = d.ct_gap[cb + c];
      finish(d, r, 0, it, rn);
      return;
    }
    if (it >= d.max_newton) {
      finish(d, r, 1, it, rn);
      return;
    }
  }
  __syncthreads();
  if (lane == 0) {
    d.st_rhs[5 * r] += 1 + nc;                      // right-hand sides
    d.st_rhs[5 * r + 1] += min(1 + nc, NT);         // forward-swept inside the factorisation
    // column passes of the substitution and the contact products they form (none without
    // contacts), and the steps with contacts
    d.st_rhs[5 * r + 2] += nc > 0 ? (1 + nc + NT - 1) / NT : 0;
    d.st_rhs[5 * r + 3] += (int64_t)(1 + nc) * nc;
    d.st_rhs[5 * r + 4] += nc > 0 ? 1 : 0;
  }

  // ---------------------------------------------------------------- right-hand side
  double* Zr = d.Z + d.zoff[r];
  const int64_t b0 = 0;                 // base node g = o
  const double bd[3] = {d.base_dir[3 * r], d.base_dir[3 * r + 1], d.base_dir[3 * r + 2]};
  double dx0[3];
  {
    const double dep = d.depth_cur[r];
    for (int k = 0; k < 3; ++k) dx0[k] = d.base_pos[3 * r + k] + dep * bd[k] - d.X[k * N + o + b0];
  }
  // col 0 = -F over free DOFs (Z's column 0).  The contact columns 1 + c (n_c at the contact
  // node, zero elsewhere) are never stored: the forward sweeps generate them.
  for (int64_t f = lane; f < nf; f += NT) {
    const int64_t g = o + f + 1;
    for (int k = 0; k < 6; ++k) Zr[6 * f + k] = -d.F[k * N + g];
  }
  // prescribed increments: base coupling into node 1, guided lateral DOFs
  if (lane == 0) {
    // rows of node 1 (f = 0): -= K[1,0] dx0 = S_0^T dx0 (S_0 = K[0,1], the base element's K_ab)
    const ElemK K0 = load_elem(d, o);
    for (int a = 0; a < 6; ++a) {
      double s = 0.0;
      for (int b = 0; b < 3; ++b) s += k_ab(K0, b, a) * dx0[b];
      Zr[a] -= s;
    }
  }
  __syncthreads();
  // guided nodes: rhs -= K xp over the block-tridiagonal neighbourhood, then rhs = xp
  {
    // xp at node i (free index f = i-1), lateral DOFs only
    for (int64_t f = lane; f < nf; f += NT) {
      const int64_t i = f + 1;
      double acc[6] = {0, 0, 0, 0, 0, 0};
      bool any = false;
      if (!G.dof(i - 1, 0) && !G.dof(i - 1, 1) && !G.dof(i - 1, 2) && !G.dof(i, 0) && !G.dof(i, 1) &&
          !G.dof(i, 2) && (i + 1 >= n || (!G.dof(i + 1, 0) && !G.dof(i + 1, 1) && !G.dof(i + 1, 2))))
        continue;
      const ElemK KL = load_elem(d, o + i - 1);                 // element (i-1, i)
      const ElemK KR = load_elem(d, o + (i + 1 < n ? i : i - 1));  // element (i, i+1) if any
      for (int64_t jn = i - 1; jn <= i + 1; ++jn) {
        if (jn < 1 || jn >= n) continue;
        for (int k = 0; k < 3; ++k) {
          if (!G.dof(jn, k)) continue;
          const double xp = d.base_pos[3 * r + k] - d.X[k * N + o + jn];
          any = true;
          for (int a = 0; a < 6; ++a) {
            double kij;
            if (jn == i) kij = k_bb(KL, a, k) + (i + 1 < n ? k_aa(KR, a, k) : 0.0);
            else if (jn == i + 1) kij = k_ab(KR, a, k);          // K[i, i+1]
            else kij = k_ab(KL, k, a);                           // K[i, i-1] = K[i-1, i]^T
            acc[a] += kij * xp;
          }
        }
      }
      if (any) {
        for (int a = 0; a < 6; ++a) Zr[6 * f + a] -= acc[a];
      }
    }
  }
  __syncthreads();
  for (int64_t f = lane; f < nf; f += NT) {
    const int64_t i = f + 1;
    for (int k = 0; k < 3; ++k)
      if (G.dof(i, k)) Zr[6 * f + k] = d.base_pos[3 * r + k] - d.X[k * N + o + i];
  }
  __syncthreads();
}

// 1/sqrt(x) for x > 0: the hardware estimate refined by two Newton steps
// y <- y + y (1/2 - x y^2 / 2) (quadratic convergence from ~23 correct bits to full FP64)
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = fma(y, fma(-h * y, y, 0.5), y);
  y = fma(y, fma(-h * y, y, 0.5), y);
  return y;
}

// phase 2: block-tridiagonal Cholesky of the QP tangent, eliminated from both ends, with the
// forward substitution of the first NT right-hand sides running one node behind it.
// The free nodes 0 .. m-1 are eliminated from the base and nf-1 .. m+1 from the tip
// (m = nf / 2), the middle node m last: the Cholesky factorisation K = L L^T in the node
// order 0, 1, .., m-1, nf-1, .., m+1, m, whose serial chain is half as long.
// Four wavefronts per robot: per side, one factors and one sweeps forward.  The factoring
// wave takes one node per step; per node, lane L < 36 owns entry (a, b) = (L / 6, L % 6):
//   per chunk of CHF steps, lane u generates step u's blocks D_i and the coupling C = K[i, next]
//   to the node eliminated next on its side (i+1 from the base, i-1 from the tip) from the
//   chord directions and constants of the node's two elements (prefetched into registers during
//   the previous chunk) and stages them in LDS;
//   A = D_i - X_prev X_prev^T  (X_prev = the previous step's coupling block; row a kept in
//   registers, row b read from LDS)
//   every lane reads A's lower triangle from LDS and factors it in registers (right-looking,
//   reciprocal square roots only), L_ii = chol(A);  row a of X = L[next, i] solves L_ii x = C[:, a].
// LD holds L_ii with the reciprocal of its diagonal, LS the block X of every node but the
// middle one (its coupling towards the middle).  The middle node's pivot block takes both
// sides' Schur complements, A_m = D_m - X_top X_top^T - X_bot X_bot^T.  Rows and columns of
// prescribed DOFs are replaced by the identity.  Both sides take the same number of steps
// (the shorter idles) so that the barriers match.
// The factoring wave also puts L_ii and X into small LDS rings; between the same two barriers
// of step k, its side's forward wave (one lane per right-hand side) takes step k-1,
// y = L_ii^-1 (b - X_prev y_prev), from the rings, reading b of column 0 from Z and generating
// the contact columns (n_c at the contact node; (1 - s) n_c and s n_c at the two nodes of a
// contact along an element), and keeps y at the checkpoint nodes in Y.
// At the middle node the forward values of both sides meet: z_m = L_m^-1 (b_m - X_top y_top -
// X_bot y_bot), and the middle node's solution x_m = L_m^-T z_m goes to XM, where the
// substitution starts both sides' backward sweeps.
__global__ void __launch_bounds__(4 * NT) __attribute__((amdgpu_waves_per_eu(3))) factor_kernel(Dev d) {
  if ((int)blockIdx.x >= d.wl_cnt[WL_ACT]) return;
  const int r = d.wl[WL_ACT * d.B + blockIdx.x];   // longest robots first
  const int w = threadIdx.x / NT, lane = threadIdx.x % NT;
  const int sd = w >> 1;                      // side: 0 from the base, 1 from the tip
  const bool fw = (w & 1) != 0;               // the side's forward-substitution wave
  if (d.st_done[r]) return;
  const int64_t o = d.off[r], n = d.off[r + 1] - o;
  const int64_t nf = n - 1;
  const Guide G = make_guide(d, r, n);
  const int64_t m = nf / 2;                   // the middle free node
  const int64_t cnt = (sd == 0) ? m : nf - 1 - m;   // this side's eliminations before the middle
  const int64_t K = m;                        // steps (the tip side has m or m - 1)
  __shared__ double sKD[2][CHF * 36], sKS[2][CHF * 36];
  __shared__ double sA[2][36], sX[2][36];
  __shared__ double rD[2][2][36], rS[2][3][36];   // L_ii by step % 2, X by step % 3, per side
  __shared__ int32_t sFC[NT];
  __shared__ double sNC[3 * NT];
  __shared__ double sSC[NT];                  // contact column's s (row on nodes fc, fc + 1)
  __shared__ double sYB[6 * NT];              // the tip side's last forward values
  __shared__ double sLm[36];
  __shared__ int s_fail;
  const int la = lane < 36 ? lane : 35;       // lanes 36..63 mirror lane 35 (results unused)
  const int a = la / 6, b = la % 6;
  double Xa[6] = {0, 0, 0, 0, 0, 0};          // row a of X_prev
  if (!fw && lane < 36) sX[sd][lane] = 0.0;
  if (threadIdx.x == 0) s_fail = 0;
  bool fail = false;
  // free index of this side's k-th elimination; node i = f + 1 has elements o+f and o+f+1
  auto fidx = [&](int64_t k) { return sd == 0 ? k : nf - 1 - k; };
  // forward waves: right-hand side `lane` (column c); column 0 is read from Z, contact column
  // 1 + c is n_c at free node fc, zero elsewhere (kept in LDS: registers live across the loop
  // also count against the factoring waves)
  const int ncol = 1 + d.st_nc[r];
  const bool col = fw && lane < ncol;
  const int64_t zp = d.zp;
  double* z = d.Y + 6 * o * zp + (col ? lane : 0);   // column `lane` of Y: row 6 j + q at z[(6j+q)*zp]
  const double* z0 = d.Z + d.zoff[r];                // column 0's right-hand side (Z, contiguous)
  if (w == 1) {
    int32_t fc = -1;
    double n0 = 0.0, n1 = 0.0, n2 = 0.0, sv = 0.0;
    if (col && lane > 0) {
      const int64_t cb = (int64_t)r * d.cap + (lane - 1);
      fc = d.ct_node[cb] - 1;
      n0 = d.ct_n[3 * cb]; n1 = d.ct_n[3 * cb + 1]; n2 = d.ct_n[3 * cb + 2];
      sv = d.ct_s[cb];
    }
    sFC[lane] = fc;
    sNC[lane] = n0; sNC[NT + lane] = n1; sNC[2 * NT + lane] = n2;
    sSC[lane] = sv;
  }
  __syncthreads();
  double yp[6] = {0, 0, 0, 0, 0, 0}, zn[6] = {0, 0, 0, 0, 0, 0};
  auto rhs = [&](int64_t j, double* v) {      // b of free node j
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < 6; ++q) v[q] = col ? z0[6 * j + q] : 0.0;
    } else {
      // the row's weight at node j: 1 - s at the contact node, s at the next one
      const int64_t fcl = sFC[lane];
      const double sv = sSC[lane];
      const double wgt = j == fcl ? 1.0 - sv : ((sv > 0.0 && j == fcl + 1) ? sv : 0.0);
      v[0] = wgt * sNC[lane]; v[1] = wgt * sNC[NT + lane];
      v[2] = wgt * sNC[2 * NT + lane];
      v[3] = 0.0; v[4] = 0.0; v[5] = 0.0;
    }
  };
  auto fwd_load = [&](int64_t k) {
    if (k < cnt) {
      rhs(fidx(k), zn);
    } else {
#pragma unroll
      for (int q = 0; q < 6; ++q) zn[q] = 0.0;
    }
  };
  auto fwd_step = [&](int64_t k) {            // forward substitution at this side's step k
    const int64_t j = fidx(k);
    double bv[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) bv[q] = zn[q];
    fwd_load(k + 1);
    if (k > 0) {
      const double* Ls = rS[sd][(k - 1) % 3];  // the previous step's X
#pragma unroll
      for (int p = 0; p < 6; ++p)
#pragma unroll
        for (int q = 0; q < 6; ++q) bv[p] -= Ls[p * 6 + q] * yp[q];
    }
    const double* Ld = rD[sd][k % 2];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const double y = bv[q] * Ld[q * 7];
      yp[q] = y;
#pragma unroll
      for (int p = q + 1; p < 6; ++p) bv[p] -= Ld[p * 6 + q] * y;
    }
    if (col && checkpoint_node(sd == 1, j)) {
#pragma unroll
      for (int q = 0; q < 6; ++q) z[(6 * j + q) * zp] = yp[q];
    }
  };
  if (fw) fwd_load(0);
  // lane u < CHF of a factoring wave prefetches the two elements of its side's step k0 + u
  ElemK pL, pR;
  bool pr = false;
  auto fetch = [&](int64_t k0) {
    const int64_t k = k0 + lane;
    if (!fw && lane < CHF && k < cnt) {
      const int64_t f = fidx(k);
      pL = load_elem(d, o + f);
      pr = f + 1 < nf;
      pR = load_elem(d, o + (pr ? f + 1 : f));
    }
  };
  fetch(0);
  for (int64_t k0 = 0; k0 < K; k0 += CHF) {
    __syncthreads();
    if (!fw && lane < CHF && k0 + lane < cnt) {
      double* D = sKD[sd] + lane * 36;
      double* C = sKS[sd] + lane * 36;
#pragma unroll
      for (int row = 0; row < 6; ++row)
#pragma unroll
        for (int cl = 0; cl < 6; ++cl) {
          D[row * 6 + cl] = k_bb(pL, row, cl) + (pr ? k_aa(pR, row, cl) : 0.0);
          // K[i, i+1] = K_ab of the right element; K[i, i-1] = K_ab of the left one, transposed
          C[row * 6 + cl] = (sd == 0) ? k_ab(pR, row, cl) : k_ab(pL, cl, row);
        }
    }
    __syncthreads();
    if (k0 + CHF < K) fetch(k0 + CHF);
    const int64_t k1 = min(K, k0 + CHF);
    for (int64_t k = k0; k < k1; ++k) {
      const bool act = k < cnt;
      const int64_t f = fidx(k), i = f + 1, g = o + i;
      const int64_t inext = (sd == 0) ? i + 1 : i - 1;
      const int lf = (int)(k - k0) * 36;
      double sc[6];
      if (!fw && act) {
        double dv = sKD[sd][lf + la];
        if (G.dof(i, a) || G.dof(i, b)) dv = (a == b) ? 1.0 : 0.0;
        // A(a, b) = D(a, b) - X_prev[a,:] . X_prev[b,:]
        double acc = dv;
#pragma unroll
        for (int q = 0; q < 6; ++q) acc -= Xa[q] * sX[sd][b * 6 + q];
        if (lane < 36) sA[sd][lane] = acc;
        // column a of the coupling to the next node, prescribed rows and columns removed
#pragma unroll
        for (int j = 0; j < 6; ++j) {
          double v = sKS[sd][lf + j * 6 + a];
          if (G.dof(i, j) || G.dof(inext, a)) v = 0.0;
          sc[j] = v;
        }
      }
      __syncthreads();
      if (!fw) {
        if (act) {
          double Lm[21];
#pragma unroll
          for (int p = 0, q = 0; p < 6; ++p)
#pragma unroll
            for (int c = 0; c <= p; ++c, ++q) Lm[q] = sA[sd][p * 6 + c];
          // right-looking Cholesky: scale column q, update the trailing lower triangle
          double rd[6];
#pragma unroll
          for (int q = 0; q < 6; ++q) {
            double dq = Lm[q * (q + 1) / 2 + q];
            if (!(dq > 0.0)) { fail = true; dq = 1.0; }
            const double rq = rsqrt_nr(dq);
            rd[q] = rq;
#pragma unroll
            for (int p = q + 1; p < 6; ++p) Lm[p * (p + 1) / 2 + q] *= rq;
#pragma unroll
            for (int p = q + 1; p < 6; ++p) {
              const int pp = p * (p + 1) / 2;
#pragma unroll
              for (int t = q + 1; t <= p; ++t) Lm[pp + t] -= Lm[pp + q] * Lm[t * (t + 1) / 2 + q];
            }
          }
          // row a of X: forward substitution L x = C[:, a] (right-looking)
#pragma unroll
          for (int q = 0; q < 6; ++q) {
            const double x = sc[q] * rd[q];
            Xa[q] = x;
#pragma unroll
            for (int p = q + 1; p < 6; ++p) sc[p] -= Lm[p * (p + 1) / 2 + q] * x;
          }
          // select this lane's entries with compile-time indices (keeps the arrays in registers)
          double lv = 0.0, xv = 0.0;
#pragma unroll
          for (int p = 0, q = 0; p < 6; ++p) {
#pragma unroll
            for (int c = 0; c <= p; ++c, ++q)
              if (p == a && c == b) lv = (p == c) ? rd[p] : Lm[q];   // reciprocal on the diagonal
            if (p == b) xv = Xa[p];
          }
          if (lane < 36) {
            d.LD[g * 36 + lane] = lv;
            d.LS[g * 36 + lane] = xv;
            sX[sd][lane] = xv;                                       // X[a][b] for the next node
            rD[sd][k % 2][lane] = lv;
            rS[sd][k % 3][lane] = xv;
          }
        }
      } else if (k > 0 && k - 1 < cnt) {
        fwd_step(k - 1);
      }
      __syncthreads();
    }
  }
  // the side whose last step was the loop's last still has its forward step pending
  if (fw && cnt == K && K > 0) fwd_step(K - 1);
  // ---------------------------------------------------------------- middle node
  const int64_t im = m + 1, gm = o + im;
  if (w == 0) {
    // A_m = D_m - X_top X_top^T - X_bot X_bot^T (a zero X when a side is empty)
    const bool rm = m + 1 < nf;
    const ElemK KL = load_elem(d, o + m), KR = load_elem(d, o + (rm ? m + 1 : m));
    double dv = k_bb(KL, a, b) + (rm ? k_aa(KR, a, b) : 0.0);
    if (G.dof(im, a) || G.dof(im, b)) dv = (a == b) ? 1.0 : 0.0;
    double acc = dv;
#pragma unroll
    for (int q = 0; q < 6; ++q)
      acc -= sX[0][a * 6 + q] * sX[0][b * 6 + q] + sX[1][a * 6 + q] * sX[1][b * 6 + q];
    if (lane < 36) sA[0][lane] = acc;
  } else if (w == 3) {
#pragma unroll
    for (int q = 0; q < 6; ++q) sYB[q * NT + lane] = yp[q];
  }
  __syncthreads();
  if (w == 0) {
    double Lm[21];
#pragma unroll
    for (int p = 0, q = 0; p < 6; ++p)
#pragma unroll
      for (int c = 0; c <= p; ++c, ++q) Lm[q] = sA[0][p * 6 + c];
    double rd[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      double dq = Lm[q * (q + 1) / 2 + q];
      if (!(dq > 0.0)) { fail = true; dq = 1.0; }
      const double rq = rsqrt_nr(dq);
      rd[q] = rq;
#pragma unroll
      for (int p = q + 1; p < 6; ++p) Lm[p * (p + 1) / 2 + q] *= rq;
#pragma unroll
      for (int p = q + 1; p < 6; ++p) {
        const int pp = p * (p + 1) / 2;
#pragma unroll
        for (int t = q + 1; t <= p; ++t) Lm[pp + t] -= Lm[pp + q] * Lm[t * (t + 1) / 2 + q];
      }
    }
    double lv = 0.0;
#pragma unroll
    for (int p = 0, q = 0; p < 6; ++p)
#pragma unroll
      for (int c = 0; c <= p; ++c, ++q)
        if (p == a && c == b) lv = (p == c) ? rd[p] : Lm[q];
    if (lane < 36) {
      d.LD[gm * 36 + lane] = lv;
      sLm[lane] = lv;
    }
  }
  __syncthreads();
  if (w == 1) {
    // z_m = L_m^-1 (b_m - X_top y_top - X_bot y_bot), then x_m = L_m^-T z_m into Z
    double bv[6];
    rhs(m, bv);
#pragma unroll
    for (int p = 0; p < 6; ++p)
#pragma unroll
      for (int q = 0; q < 6; ++q)
        bv[p] -= sX[0][p * 6 + q] * yp[q] + sX[1][p * 6 + q] * sYB[q * NT + lane];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const double y = bv[q] * sLm[q * 7];
      bv[q] = y;
#pragma unroll
      for (int p = q + 1; p < 6; ++p) bv[p] -= sLm[p * 6 + q] * y;
    }
    double xm[6];
#pragma unroll
    for (int q = 5; q >= 0; --q) {
      const double x = bv[q] * sLm[q * 7];
      xm[q] = x;
#pragma unroll
      for (int p = 0; p < q; ++p) bv[p] -= sLm[q * 6 + p] * x;
    }
    if (col) {
      double* zx = d.XM + ((int64_t)r * NT + lane) * 6;
#pragma unroll
      for (int q = 0; q < 6; ++q) zx[q] = xm[q];
    }
  }
  if (fail) s_fail = 1;
  __syncthreads();
  if (s_fail) finish(d, r, 3, d.st_it[r], d.st_rn[r]);
}

// phase 3: substitution of all right-hand sides with the two-ended factor of phase 2, kept
// only where the LCP needs it: the contact products W[i, c] = n_i . x_c(node of i) of every
// column c (column 0 = the free increment dx_free, 1 + j = Z_j = K^-1 A^T e_j).
// One lane per right-hand side, each lane holding its column's 6-vector.  Backward sweeps run
// from the middle node outwards: on the base side x_f = L_f^-T (y_f - X_f^T x_{f+1}) for f =
// m-1 .. f_lo, on the tip side x_f = L_f^-T (y_f - X_f^T x_{f-1}) for f = m+1 .. f_hi (X_f, the
// block stored with node f, couples it towards the middle; f_lo and f_hi are the outermost
// contact nodes, beyond which no product is needed), starting from the middle node's x_m.
// Per chunk of CHS nodes (aligned at multiples of CHS) the factor blocks are staged through
// LDS (broadcast to all lanes), the next chunk's blocks in flight in registers meanwhile; the
// chunk's forward values are recomputed from the checkpoint before it (b of column 0 read
// from Z, the contact columns generated), then swept back, and at each contact node the
// lanes write that contact's row of products (contiguous over the wavefront's columns).
// One block per robot and pass of NT columns, one wavefront per side; the two meet only at the
// middle node (each stages its own blocks).  The first NT columns were swept forward in phase
// 2, which also wrote x_m: their block only sweeps back.  Columns
// from NT on are contact columns (n_c at the contact node, zero elsewhere): their block sweeps
// them forward (generating the right-hand side, over the part of each side that the contact
// node reaches, keeping the checkpoints), combines the two sides at the middle node, then
// sweeps back.

// LDS staged by the lanes of a wavefront for itself: a wavefront's LDS operations take effect
// in order, so keeping the compiler from moving them across this point is enough
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// chunks of CHS nodes (aligned at multiples of CHS) between nodes f_a <= f_b, 0 if f_a > f_b
__device__ __forceinline__ int64_t chunk_span(int64_t f_a, int64_t f_b) {
  return f_a > f_b ? 0 : f_b / CHS - f_a / CHS + 1;
}

// first index of the robot's contact list (sorted by node) whose free node is >= f
__device__ __forceinline__ int first_contact_at(const int32_t* node, int nc, int64_t f) {
  int lo = 0, hi = nc;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if ((int64_t)node[mid] - 1 < f) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// the lane's column: right-hand side generation and the contact rows it writes
struct SweepCol {
  bool act;               // the lane holds a column
  bool col0;              // column 0: right-hand side b from Z
  int c;                  // column index
  int64_t fcn;            // contact column: its contact's free node ...
  int64_t fhi;            // ... and the last node of its row (fcn + 1 along an element)
  double cn0, cn1, cn2;   // and normal
  double cs;              // along an element: the row is (1 - s) n at fcn, s n at fcn + 1
  const double* zb;       // column 0's b (Z), NULL in blocks without column 0
  const double* yv;       // the column in Y (checkpoints)
  int64_t zp;
  const int32_t* node;    // the robot's contact list
  const double* nrm;
  const double* s;
  double* W;              // the robot's rows of contact products
  int nc;
  // the right-hand side's translation component k at free node f (contact columns)
  __device__ __forceinline__ double gen(int64_t f, int k) const {
    const double nk = k == 0 ? cn0 : (k == 1 ? cn1 : cn2);
    if (!act || k >= 3) return 0.0;
    if (f == fcn) return (1.0 - cs) * nk;
    return (cs > 0.0 && f == fcn + 1) ? cs * nk : 0.0;
  }
  // W[i, c] = (1 - s_i) n_i . x(node of i) + s_i n_i . x(next node): xa at the contact's node,
  // xb at the next one (unused for a node contact)
  __device__ __forceinline__ void put(int i, const double (&xa)[6], const double (&xb)[6]) const {
    if (!act) return;
    const double si = s[i];
    const double* ni = nrm + 3 * i;
    double v = (1.0 - si) * (ni[0] * xa[0] + ni[1] * xa[1] + ni[2] * xa[2]);
    if (si > 0.0) v += si * (ni[0] * xb[0] + ni[1] * xb[1] + ni[2] * xb[2]);
    W[(int64_t)i * zp + c] = v;
  }
};

// the contact rows completed at free node f, contacts i in sweep order.  Base side (f
// descending, x the solution at f, xp the one at f + 1): the contacts of node f.  Tip side (f
// ascending, xp the solution at f - 1): the node contacts of node f and the contacts along the
// element f-1 -> f (sorted last at node f-1, so they come first).
template <bool UP>
__device__ __forceinline__ void write_rows(const SweepCol& sc, int64_t f, int& ci, const double (&x)[6],
                                           const double (&xp)[6]) {
  if (UP) {
    while (ci < sc.nc) {
      const int64_t fi = (int64_t)sc.node[ci] - 1;
      if (fi == f - 1 && sc.s[ci] > 0.0) sc.put(ci, xp, x);
      else if (fi == f && !(sc.s[ci] > 0.0)) sc.put(ci, x, x);
      else break;
      ++ci;
    }
  } else {
    while (ci >= 0 && (int64_t)sc.node[ci] - 1 == f) {
      sc.put(ci, x, xp);
      --ci;
    }
  }
}

// backward sweep of one side; UP: f = f_begin .. f_end ascending (tip side), else f = f_begin ..
// f_end descending (base side).  ci: the first contact the side meets (tip side: the first at
// a node >= f_begin; base side: the last at a node <= f_begin).  sKD, sKS, sB: the wavefront's
// own staging arrays (sB: column 0's right-hand side of a chunk, CHS * 6 doubles).
template <bool UP>
__device__ void bwd_side(const Dev& d, int64_t o, int64_t nf, int64_t f_begin, int64_t f_end,
                         const SweepCol& sc, int ci, double (&xn)[6], double* sKD, double* sKS,
                         double* sB) {
  const int lane = threadIdx.x % NT;
  // staged per chunk [f0, f0 + CHS): LD of its nodes at u = 0..CHS-1, LS of nodes f0 - 1 + u
  // (base side) or f0 + u (tip side) at u = 0..CHS (the forward sweep's coupling to the
  // previous node and the backward sweep's coupling towards the middle), column 0's b
  double pd[PFS], ps[PFS], pb;
  auto stageK = [&]() {
#pragma unroll
    for (int u = 0; u < PFS; ++u) { sKD[lane + u * NT] = pd[u]; sKS[lane + u * NT] = ps[u]; }
    if (lane < CHS * 6) sB[lane] = pb;
  };
  auto fetchK = [&](int64_t ch) {
    const int64_t f0 = ch * CHS;
    const int64_t s0 = UP ? f0 : f0 - 1;             // first node of the LS blocks
#pragma unroll
    for (int u = 0; u < PFS; ++u) {
      const int64_t idx = lane + (int64_t)u * NT;
      const int64_t fd = f0 + idx / 36, fs = s0 + idx / 36;
      pd[u] = (idx < CHS * 36 && fd < nf) ? d.LD[(o + 1 + fd) * 36 + idx % 36] : 0.0;
      ps[u] = (idx < (CHS + 1) * 36 && fs >= 0 && fs < nf) ? d.LS[(o + 1 + fs) * 36 + idx % 36] : 0.0;
    }
    pb = (sc.zb && lane < CHS * 6 && f0 + lane / 6 < nf) ? sc.zb[6 * f0 + lane] : 0.0;
  };
  // the lane's forward value at the checkpoint before chunk ch (zero before its contact node)
  auto loadCk = [&](double (&cp)[6], int64_t ch) {
    const int64_t f0 = ch * CHS;
    const int64_t cpn = UP ? f0 + CHS : f0 - 1;
    const bool valid = sc.act && cpn >= 0 && cpn < nf &&
                       (sc.col0 || (UP ? cpn <= sc.fhi : cpn >= sc.fcn));
#pragma unroll
    for (int k = 0; k < 6; ++k) cp[k] = valid ? sc.yv[(6 * cpn + k) * sc.zp] : 0.0;
  };
  double zz[CHS * 6];                               // the chunk's forward values
  // forward values of the chunk's nodes on this side from the checkpoint
  auto recompute = [&](const double (&cp)[6], int64_t ch) {
    const int64_t f0 = ch * CHS;
    double yp[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) yp[k] = cp[k];
    auto fnode = [&](int u, int us, int64_t f) {    // us: staged LS index of the previous node
      double bv[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) bv[k] = sc.col0 ? sB[u * 6 + k] : sc.gen(f, k);
      const double* Ls = sKS + us * 36;
#pragma unroll
      for (int p = 0; p < 6; ++p)
#pragma unroll
        for (int k = 0; k < 6; ++k) bv[p] -= Ls[p * 6 + k] * yp[k];
      const double* Ld = sKD + u * 36;
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const double y = bv[k] * Ld[k * 7];
        yp[k] = y;
        zz[u * 6 + k] = y;
#pragma unroll
        for (int p = k + 1; p < 6; ++p) bv[p] -= Ld[p * 6 + k] * y;
      }
    };
    if (UP) {
#pragma unroll
      for (int u = CHS - 1; u >= 0; --u) {
        const int64_t f = f0 + u;
        if (f < nf && f >= f_begin) fnode(u, u + 1, f);
      }
    } else {
#pragma unroll
      for (int u = 0; u < CHS; ++u) {
        const int64_t f = f0 + u;
        if (f <= f_begin) fnode(u, u, f);
      }
    }
  };
  auto bnode = [&](int u, int us, int64_t f) {
    double bv[6], xp[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) { bv[k] = zz[u * 6 + k]; xp[k] = xn[k]; }
    const double* Ls = sKS + us * 36;                      // X_f: b -= X_f^T x_neighbour
#pragma unroll
    for (int k = 0; k < 6; ++k)
#pragma unroll
      for (int p = 0; p < 6; ++p) bv[p] -= Ls[k * 6 + p] * xn[k];
    const double* Ld = sKD + u * 36;
#pragma unroll
    for (int k = 5; k >= 0; --k) {
      const double x = bv[k] * Ld[k * 7];
      xn[k] = x;
#pragma unroll
      for (int p = 0; p < k; ++p) bv[p] -= Ld[k * 6 + p] * x;
    }
    write_rows<UP>(sc, f, ci, xn, xp);
  };
  auto backward = [&](int64_t ch) {
    const int64_t f0 = ch * CHS;
    if (UP) {
#pragma unroll
      for (int u = 0; u < CHS; ++u) {
        const int64_t f = f0 + u;
        if (f >= f_begin && f <= f_end) bnode(u, u, f);
      }
    } else {
#pragma unroll
      for (int u = CHS - 1; u >= 0; --u) {
        const int64_t f = f0 + u;
        if (f <= f_begin && f >= f_end) bnode(u, u + 1, f);
      }
    }
  };
  const int64_t mine = UP ? chunk_span(f_begin, f_end) : chunk_span(f_end, f_begin);
  const int64_t ch_first = f_begin / CHS;
  const int64_t step = UP ? 1 : -1;
  double ca[6], cb2[6];
  if (mine > 0) {
    fetchK(ch_first);
    loadCk(ca, ch_first);
  }
  // two chunks per pass of the loop so that the two checkpoint buffers keep fixed registers
  for (int64_t t = 0; t < mine; t += 2) {
    const int64_t ch = ch_first + t * step;
    wave_sync();
    stageK();
    wave_sync();
    if (t + 1 < mine) {
      fetchK(ch + step);
      loadCk(cb2, ch + step);
    }
    recompute(ca, ch);
    backward(ch);
    if (t + 1 >= mine) break;
    wave_sync();
    stageK();
    wave_sync();
    if (t + 2 < mine) {
      fetchK(ch + 2 * step);
      loadCk(ca, ch + 2 * step);
    }
    recompute(cb2, ch + step);
    backward(ch + step);
  }
}

// block (r, p) takes columns p*NT .. p*NT + NT-1: wave 0 the base side, wave 1 the tip side
__global__ void __launch_bounds__(2 * NT) subst_kernel(Dev d) {
  if ((int)blockIdx.x >= d.wl_cnt[WL_SUB]) return;
  const int item = d.wl_sub[blockIdx.x];     // a pass of a robot with contacts, longest first
  const int r = item & 0xffffff;
  const int w = threadIdx.x / NT, lane = threadIdx.x % NT;
  if (d.st_done[r]) return;
  const int nc = d.st_nc[r];
  if (nc == 0) return;                   // no contact: no product is needed
  const int ncol = 1 + nc;
  const int c0 = (item >> 24) * NT;
  if (c0 >= ncol) return;
  const int64_t o = d.off[r], n = d.off[r + 1] - o;
  const int64_t nf = n - 1, m = nf / 2;
  const int c = c0 + lane;
  const int64_t cb = (int64_t)r * d.cap;
  const int64_t zp = d.zp;
  SweepCol sc;
  sc.act = c < ncol;
  sc.col0 = c == 0;
  sc.c = sc.act ? c : 0;
  sc.fcn = -1;
  sc.fhi = -1;
  sc.cn0 = sc.cn1 = sc.cn2 = 0.0;
  sc.cs = 0.0;
  sc.zb = c0 == 0 ? d.Z + d.zoff[r] : nullptr;   // column 0's b (the first block only)
  sc.zp = zp;
  sc.yv = d.Y + 6 * o * zp + sc.c;
  sc.node = d.ct_node + cb;
  sc.nrm = d.ct_n + 3 * cb;
  sc.s = d.ct_s + cb;
  sc.W = d.W + cb * zp;
  sc.nc = nc;
  double* yv = d.Y + 6 * o * zp + sc.c;
  __shared__ double sKD[2][PFS * NT], sKS[2][PFS * NT];
  __shared__ double sXT[6 * NT], sXM[6 * NT], sB[2][CHS * 6];
  const bool fwd = c0 > 0;                // the first NT columns were swept forward in phase 2
  if (sc.act && c > 0) {
    const int64_t ci = cb + (c - 1);
    sc.fcn = d.ct_node[ci] - 1;
    sc.cn0 = d.ct_n[3 * ci]; sc.cn1 = d.ct_n[3 * ci + 1]; sc.cn2 = d.ct_n[3 * ci + 2];
    sc.cs = d.ct_s[ci];
    sc.fhi = sc.fcn + (sc.cs > 0.0 ? 1 : 0);
  }
  // ---------------------------------------------------------------- forward sweeps
  // base side: f = fs .. m-1 ascending, b - X_{f-1} y_{f-1}; tip side: f = fe .. m+1
  // descending, b - X_{f+1} y_{f+1}; a side's values are zero before the contact node
  double yp[6] = {0, 0, 0, 0, 0, 0};
  if (fwd) {
    double* KD = sKD[w];
    double* KS = sKS[w];
    double pd[PFS], ps[PFS];
    const bool up = w == 0;
    const int64_t fcn = sc.fcn;
    const bool act = sc.act;
    int64_t lim;                          // first (base side) / last (tip side) row node
    {
      long long v = act ? (up ? fcn : sc.fhi) : (up ? (long long)nf : -1ll);
#pragma unroll
      for (int sh = 32; sh > 0; sh >>= 1) {
        const long long ov = __shfl_xor(v, sh);
        v = up ? min(v, ov) : max(v, ov);
      }
      lim = v;
    }
    // chunk [f0, f0+CHS): LD of its nodes and, per node, X of the previous node in sweep order
    auto fetchF = [&](int64_t f0) {
      const int64_t cnt = min((int64_t)CHS, nf - f0) * 36;
      const int64_t sh = up ? -1 : 1;
      const double* ldp = d.LD + (o + 1 + f0) * 36;
      const double* lsp = d.LS + (o + 1 + f0 + sh) * 36;
#pragma unroll
      for (int u = 0; u < PFS; ++u) {
        const int64_t idx = lane + (int64_t)u * NT;
        const int64_t fn = f0 + idx / 36 + sh;        // the neighbour whose block is read
        pd[u] = idx < cnt ? ldp[idx] : 0.0;
        ps[u] = (idx < cnt && fn >= 0 && fn < nf) ? lsp[idx] : 0.0;
      }
    };
    auto fnode = [&](int u, int64_t f) {
      double bv[6] = {sc.gen(f, 0), sc.gen(f, 1), sc.gen(f, 2), 0.0, 0.0, 0.0};
      const double* Ls = KS + u * 36;
#pragma unroll
      for (int p = 0; p < 6; ++p)
#pragma unroll
        for (int k = 0; k < 6; ++k) bv[p] -= Ls[p * 6 + k] * yp[k];
      const double* Ldd = KD + u * 36;
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const double y = bv[k] * Ldd[k * 7];
        yp[k] = y;
#pragma unroll
        for (int p = k + 1; p < 6; ++p) bv[p] -= Ldd[p * 6 + k] * y;
      }
      if (act && checkpoint_node(!up, f)) {
#pragma unroll
        for (int k = 0; k < 6; ++k) yv[(6 * f + k) * zp] = yp[k];
      }
    };
    // this side's nodes: base [max(lim, 0), m), tip (m, min(lim, nf-1)]
    const int64_t lo = up ? lim : m + 1;
    const int64_t hi = up ? m - 1 : lim;
    const int64_t nch_lo = lo / CHS, nch_hi = hi >= 0 ? hi / CHS : -1;
    const int64_t mine = (lo <= hi) ? nch_hi - nch_lo + 1 : 0;
    if (mine > 0) fetchF((up ? nch_lo : nch_hi) * CHS);
    for (int64_t t = 0; t < mine; ++t) {
      const int64_t ch = up ? nch_lo + t : nch_hi - t;
      wave_sync();
#pragma unroll
      for (int u = 0; u < PFS; ++u) { KD[lane + u * NT] = pd[u]; KS[lane + u * NT] = ps[u]; }
      wave_sync();
      if (t + 1 < mine) fetchF((up ? ch + 1 : ch - 1) * CHS);
      {
        const int64_t f0 = ch * CHS;
        if (up) {
#pragma unroll
          for (int u = 0; u < CHS; ++u) {
            const int64_t f = f0 + u;
            if (f >= lo && f <= hi) fnode(u, f);
          }
        } else {
#pragma unroll
          for (int u = CHS - 1; u >= 0; --u) {
            const int64_t f = f0 + u;
            if (f >= lo && f <= hi) fnode(u, f);
          }
        }
      }
    }
  }
  // ---------------------------------------------------------------- middle node
  // z_m = L_m^-1 (b_m - X_{m-1} y_{m-1} - X_{m+1} y_{m+1}), x_m = L_m^-T z_m (phase 2 wrote
  // it to XM for the first NT columns)
  if (!fwd) {
    if (w == 0) {
      const double* xm = d.XM + ((int64_t)r * NT + lane) * 6;
#pragma unroll
      for (int k = 0; k < 6; ++k) sXM[k * NT + lane] = sc.act ? xm[k] : 0.0;
    }
  } else if (w == 1) {
#pragma unroll
    for (int k = 0; k < 6; ++k) sXT[k * NT + lane] = yp[k];
  }
  __syncthreads();
  if (fwd && w == 0) {
    double bv[6] = {sc.gen(m, 0), sc.gen(m, 1), sc.gen(m, 2), 0.0, 0.0, 0.0};
    const bool ht = m >= 1, hb = m + 1 < nf;
    const double* Xt = d.LS + (o + 1 + (ht ? m - 1 : m)) * 36;   // X_{m-1} (base side), if any
    const double* Xb = d.LS + (o + 1 + (hb ? m + 1 : m)) * 36;   // X_{m+1} (tip side), if any
#pragma unroll
    for (int p = 0; p < 6; ++p)
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        if (ht) bv[p] -= Xt[p * 6 + k] * yp[k];
        if (hb) bv[p] -= Xb[p * 6 + k] * sXT[k * NT + lane];
      }
    const double* Lm = d.LD + (o + 1 + m) * 36;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const double y = bv[k] * Lm[k * 7];
      bv[k] = y;
#pragma unroll
      for (int p = k + 1; p < 6; ++p) bv[p] -= Lm[p * 6 + k] * y;
    }
#pragma unroll
    for (int k = 5; k >= 0; --k) {
      const double x = bv[k] * Lm[k * 7];
      sXM[k * NT + lane] = x;
#pragma unroll
      for (int p = 0; p < k; ++p) bv[p] -= Lm[k * 6 + p] * x;
    }
  }
  __syncthreads();
  // ---------------------------------------------------------------- backward sweeps
  double xn[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) xn[k] = sXM[k * NT + lane];
  // the outermost row nodes bound the sweeps (the list is by node, a node's contacts along
  // its element last); the middle node's own contacts take x_m, a contact along the element
  // m -> m+1 is completed by the tip side
  const int64_t f_lo = (int64_t)sc.node[0] - 1;
  const int64_t f_hi = (int64_t)sc.node[nc - 1] - 1 + (sc.s[nc - 1] > 0.0 ? 1 : 0);
  const int i_mid = first_contact_at(sc.node, nc, m);
  int i_tip = i_mid;
  while (i_tip < nc && (int64_t)sc.node[i_tip] - 1 == m && !(sc.s[i_tip] > 0.0)) ++i_tip;
  if (w == 0) {
    int ci = i_mid;
    write_rows<true>(sc, m, ci, xn, xn);
  }
  if (w == 0) bwd_side<false>(d, o, nf, m - 1, f_lo, sc, i_mid - 1, xn, sKD[0], sKS[0], sB[0]);
  else bwd_side<true>(d, o, nf, m + 1, f_hi, sc, i_tip, xn, sKD[1], sKS[1], sB[1]);
}

// phase 4: contact Schur complement, LCP, step limit and state update

constexpr int LCPM = 64;  // contact sets up to this size take the parallel LCP in LDS

__device__ __forceinline__ int pk(int i, int j) {  // packed lower-triangle index, i >= j
  return i * (i + 1) / 2 + j;
}
__device__ __forceinline__ int pks(int i, int j) {  // packed index of a symmetric entry
  return i >= j ? pk(i, j) : pk(j, i);
}

// lexicographic minimum of (v, index) over the wavefront; identical in every lane
__device__ __forceinline__ void wave_argmin(double& v, int& idx) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(v, o);
    const int oi = __shfl_xor(idx, o);
    if (ov < v || (ov == v && oi < idx)) { v = ov; idx = oi; }
  }
}

// Primal active-set method for the LCP  w = W y + q >= 0, y >= 0, y.w = 0  with W symmetric
// positive semidefinite, i.e. the convex QP  min 1/2 y.W y + q.y  over y >= 0 (the Lawson-Hanson
// scheme): add the most violated inactive constraint (most negative w), solve
// W_PP z = -q_P; if z > 0 take it, else move from y toward z until the first active y
// reaches zero, drop those and solve again.  This version runs on one wavefront for
// m <= LCPM with everything in LDS.  Lane i owns constraint i.  sW holds W packed (lower, constraint
// order); sL the Cholesky factor of W_PP packed with rows in active-set order and sRd its
// reciprocal diagonal; sP the active set in order of entry; sYp the active y by position.
// Adding the most violated constraint appends one row to the factor; one that depends
// linearly on the active set (W only semidefinite: more contacts at a node than it has
// directions) is exchanged for an active one along a null direction of W; dropping
// constraints refactors.  `warm` flags a starting active set (the contacts active at the previous
// iteration); it is used when its own solution is positive, else the start is empty.
// Returns false on a non-positive pivot, a dependent constraint that no active one can
// give way to, or when the iteration limits are reached.
struct LcpLds {
  double W[LCPM * (LCPM + 1) / 2];
  double L[LCPM * (LCPM + 1) / 2];
  double Rd[LCPM];
  double Yp[LCPM];
  double Yc[LCPM];
  double Q[LCPM];
  int P[LCPM];
  int In[LCPM];
};

// Cholesky by columns of the block gathered into the packed rows of L (np <= NT, row p on lane
// p): l_pj = (w_pj - sum_{k<j} l_pk l_jk) / l_jj, subtracting in the order k = 0, 1, ... (the
// rounding of the elimination by rows).  Software-pipelined: the sum over k < j - 1 of the
// next column is read from LDS while the pivot's reciprocal square root is formed, and the
// last term comes from registers (each lane keeps its newest entry; row j's by a lane read),
// so the serial chain per column holds no LDS access.  The diagonal keeps the pivot, Rd its
// reciprocal square root.  Returns false on a non-positive pivot.
__device__ bool chol_cols1(double* L, double* Rd, int np) {
  const int lane = threadIdx.x;
  const double* Lp = L + pk(lane, 0);            // this lane's row (read inside the triangle)
  bool ok = true;
  double part = np > 0 ? Lp[0] : 0.0;            // column 0: nothing to subtract
  double last = 0.0;                             // l_{p, j-1}
  for (int j = 0; j < np; ++j) {
    const double a = j > 0 ? part - last * lane_read(last, j) : part;
    const double piv = lane_read(a, j);
    // next column's sum over k < j (rows p and j + 1, columns finished before this one)
    double nxt = 0.0;
    if (j + 1 < np) {
      const double* Lj1 = L + pk(j + 1, 0);
      nxt = Lp[j + 1];
#pragma unroll 8
      for (int k = 0; k < j; ++k) nxt -= Lp[k] * Lj1[k];
    }
    if (!(piv > 0.0)) ok = false;
    const double rk = rsqrt_nr(piv > 0.0 ? piv : 1.0);
    const double lpj = lane == j ? a : a * rk;
    if (lane >= j && lane < np) L[pk(lane, j)] = lpj;
    if (lane == 0) Rd[j] = rk;
    last = lpj;
    part = nxt;
    __syncthreads();
  }
  return ok;
}

// Cholesky of W(P, P): the block gathered from the packed W, then factored by columns
__device__ bool lcp_factor(LcpLds& S, int np) {
  const int lane = threadIdx.x;
  // W(P, P) into the packed rows, eight reads in flight before their writes
  const int pl = lane < np ? S.P[lane] : 0;
  for (int b0 = 0; b0 < np; b0 += 8) {
    double v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int b = b0 + e < np ? b0 + e : 0;
      v[e] = S.W[pks(pl, __builtin_amdgcn_readlane(pl, b))];
    }
#pragma unroll
    for (int e = 0; e < 8; ++e)
      if (lane < np && b0 + e <= lane) S.L[pk(lane, b0 + e)] = v[e];
  }
  __syncthreads();
  return chol_cols1(S.L, S.Rd, np);
}

// Triangular solves with a packed lower factor L (rows by position, true off-diagonal entries)
// and its reciprocal diagonal Rd, position p on lane p, np <= NT.  A serial chain over the
// positions: each step takes x_k from lane k by a lane read and updates the other lanes
// without branches, the next step's Rd and L entries already in flight.  Every lane reads
// inside the packed triangle of NT rows (entries it does not use among them).
// L x = b, in place
__device__ __forceinline__ double tri_fwd1(const double* L, const double* Rd, int np, double b) {
  const int lane = threadIdx.x;
  if (np <= 0) return b;
  const double* Lr = L + pk(lane, 0);            // this lane's row: entry k at Lr[k]
  double rd = Rd[0], l = Lr[0];
  for (int k = 0; k < np; ++k) {
    const int kn = k + 1 < np ? k + 1 : k;
    const double rdn = Rd[kn], ln = Lr[kn];
    const double xk = lane_read(b, k) * rd;
    const double u = b - l * xk;
    b = lane == k ? xk : (lane > k && lane < np ? u : b);
    rd = rdn;
    l = ln;
  }
  return b;
}
// L^T x = b, in place
__device__ __forceinline__ double tri_bwd1(const double* L, const double* Rd, int np, double b) {
  const int lane = threadIdx.x;
  if (np <= 0) return b;
  double rd = Rd[np - 1], l = L[pk(np - 1, lane)];
  for (int k = np - 1; k >= 0; --k) {
    const int kn = k > 0 ? k - 1 : 0;
    const double rdn = Rd[kn], ln = L[pk(kn, lane)];
    const double xk = lane_read(b, k) * rd;
    const double u = b - l * xk;
    b = lane == k ? xk : (lane < k ? u : b);
    rd = rdn;
    l = ln;
  }
  return b;
}

// lanes a < np: solve L L^T z = b (b, z by position)
__device__ __forceinline__ double lcp_solve(const LcpLds& S, int np, double bv) {
  return tri_bwd1(S.L, S.Rd, np, tri_fwd1(S.L, S.Rd, np, bv));
}

__device__ bool lcp_parallel(LcpLds& S, const double* q, int m, bool warm, double& y_out) {
  const int lane = threadIdx.x;
  const double qi = lane < m ? q[lane] : 0.0;
  const double tolw = 1e-12 * warp_max(fabs(qi));
  int np = 0;
  if (lane < LCPM) { S.In[lane] = 0; S.Yc[lane] = 0.0; S.Q[lane] = qi; }
  __syncthreads();
  // warm start: solve on the flagged set, drop the constraints whose y is not positive and
  // solve again, until every y is positive (a feasible start) or the set is empty
  unsigned long long wm = __ballot(warm && lane < m);
  while (wm) {
    const int cnt = __popcll(wm);
    const bool mine = (wm >> lane) & 1ull;
    const int pos = __popcll(wm & ((1ull << lane) - 1ull));
    if (mine) S.P[pos] = lane;
    __syncthreads();
    if (!lcp_factor(S, cnt)) break;
    const double z = lcp_solve(S, cnt, lane < cnt ? -S.Q[S.P[lane]] : 0.0);
    const unsigned long long bad = __ballot(lane < cnt && !(z > 0.0));
    if (bad == 0ull) {
      if (lane < cnt) { S.Yp[lane] = z; S.In[S.P[lane]] = 1; }
      np = cnt;
      __syncthreads();
      break;
    }
    wm = __ballot(mine && !((bad >> pos) & 1ull));
    __syncthreads();
  }
  bool done = false, failed = false;
  for (int outer = 0; outer < 4 * m + 8 && !done && !failed; ++outer) {
    // most violated inactive constraint
    // the active set's indices and forces by lane reads: the products' loads are independent
    const int pl = lane < np ? S.P[lane] : 0;
    const double yl = lane < np ? S.Yp[lane] : 0.0;
    const int row = lane < m ? lane : 0;
    double w = qi;
#pragma unroll 4
    for (int a = 0; a < np; ++a)
      w += S.W[pks(row, __builtin_amdgcn_readlane(pl, a))] * lane_read(yl, a);
    double v = (lane < m && !S.In[lane] && w < -tolw) ? w : INFINITY;
    int t = lane;
    wave_argmin(v, t);
    if (!(v < INFINITY)) { done = true; break; }
    // append t: new factor row l solves L l = W(P, t)
    double bv = lane < np ? S.W[pks(S.P[lane], t)] : 0.0;
    bv = tri_fwd1(S.L, S.Rd, np, bv);
    const double dtt = S.W[pk(t, t)] - warp_sum(lane < np ? bv * bv : 0.0);
    __syncthreads();
    if (dtt > 0.0) {
      if (lane < np) S.L[pk(np, lane)] = bv;
      if (lane == 0) {
        S.L[pk(np, np)] = 1.0;
        S.Rd[np] = rsqrt_nr(dtt);
        S.P[np] = t;
        S.Yp[np] = 0.0;
        S.In[t] = 1;
      }
      ++np;
      __syncthreads();
    } else {
      // t depends linearly on the active set (several contacts at one node): W(P, t) =
      // W_PP c.  Raising y_t by s and lowering y_P by s c leaves every w unchanged; the
      // first active y to reach zero (smallest y_a / c_a over c_a > 0) leaves and t takes
      // its position, which keeps the set independent.  No c_a > 0: no solution.
      const double c = lcp_solve(S, np, lane < np ? S.W[pks(S.P[lane], t)] : 0.0);
      const double cmax = warp_max(lane < np ? fabs(c) : 0.0);
      double rat = (lane < np && c > 1e-12 * cmax) ? S.Yp[lane] / c : INFINITY;
      int jp = lane;
      wave_argmin(rat, jp);
      if (!(rat < INFINITY)) { failed = true; break; }
      const double yv = lane < np ? (lane == jp ? rat : fmax(S.Yp[lane] - rat * c, 0.0)) : 0.0;
      const int oldj = S.P[jp];
      __syncthreads();
      if (lane < np) S.Yp[lane] = yv;
      if (lane == 0) { S.In[oldj] = 0; S.P[jp] = t; S.In[t] = 1; }
      __syncthreads();
      if (!lcp_factor(S, np)) { failed = true; break; }
    }
    for (int inner = 0; inner < 4 * m + 8; ++inner) {
      const double z = lcp_solve(S, np, lane < np ? -S.Q[S.P[lane]] : 0.0);
      if (__ballot(lane < np && !(z > 0.0)) == 0ull) {
        if (lane < np) S.Yp[lane] = z;
        __syncthreads();
        break;
      }
      // step toward z until the first active y reaches zero
      const double yp = lane < np ? S.Yp[lane] : 0.0;
      double al = (lane < np && z <= 0.0) ? yp / (yp - z) : 1.0;
      al = fmin(1.0, warp_min(al));
      const double yn = yp + al * (z - yp);
      const bool keep = lane < np && yn > 0.0;
      const unsigned long long km = __ballot(keep);
      const int pidx = lane < np ? S.P[lane] : 0;
      __syncthreads();
      if (lane < np && !keep) S.In[pidx] = 0;
      if (keep) {
        const int pos = __popcll(km & ((1ull << lane) - 1ull));
        S.P[pos] = pidx;
        S.Yp[pos] = yn;
      }
      np = __popcll(km);
      __syncthreads();
      if (np == 0) break;
      if (!lcp_factor(S, np)) { failed = true; break; }
    }
  }
  if (failed || !done) return false;
  if (lane < np) S.Yc[S.P[lane]] = S.Yp[lane];
  __syncthreads();
  y_out = lane < m ? S.Yc[lane] : 0.0;
  return true;
}

// q_c = gap_c + n_c . dx_free(node of c) for the nc contacts of robot r (Wr: the robot's rows
// of contact products, column 0 = n_c . dx_free)
__device__ void contact_q(const Dev& d, int64_t cb, int nc, const double* Wr, double* qv) {
  for (int a = threadIdx.x; a < nc; a += NT) qv[a] = d.ct_gap[cb + a] + Wr[(int64_t)a * d.zp];
}

// After the LCP of robot r (one wavefront): the contacts with force > 0 in index order
// (y by contact index in ct_y) into ac_idx / ac_y, their count into st_nact; clears st_mx.
__device__ void store_active(const Dev& d, int r, int nc) {
  const int lane = threadIdx.x;
  const int64_t cb = (int64_t)r * d.cap;
  const double* y = d.ct_y + cb;
  int nact = 0;
  for (int i0 = 0; i0 < nc; i0 += NT) {
    const int i = i0 + lane;
    const double yi = i < nc ? y[i] : 0.0;
    const unsigned long long am = __ballot(yi > 0.0);
    if (yi > 0.0) {
      const int pos = nact + __popcll(am & ((1ull << lane) - 1ull));
      d.ac_idx[cb + pos] = i;
      d.ac_y[cb + pos] = yi;
    }
    nact += __popcll(am);
  }
  if (lane == 0) {
    d.st_nact[r] = nact;
    d.st_mx[r] = 0ull;
  }
}

// translation increment of the base node: to the clamped, inserted position (eq. 14)
__device__ __forceinline__ void base_increment(const Dev& d, int r, int64_t o, double* dx0) {
  const double dep = d.depth_cur[r];
  for (int k = 0; k < 3; ++k)
    dx0[k] = d.base_pos[3 * r + k] + dep * d.base_dir[3 * r + k] - d.X[k * d.Ntot + o];
}

// largest-translation reduction: a wavefront whose nodes all belong to robot r combines
// its candidates first; v < 0 means no candidate (NaN translations are ignored, as fmax does)
__device__ __forceinline__ void step_max(const Dev& d, int r, double v) {
  const int rf = __shfl(r, 0);
  const bool one = __ballot(r != rf) == 0ull;
  if (one) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0 && v >= 0.0)
      atomicMax(d.st_mx + r, (unsigned long long)__double_as_longlong(v));
  } else if (v >= 0.0) {
    atomicMax(d.st_mx + r, (unsigned long long)__double_as_longlong(v));
  }
}

// phase 4b of the ADMM variant, one thread per node: the robot's largest node translation of
// the step dx in Z's column 0
__global__ void __launch_bounds__(256) step_dx_kernel(Dev d) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = g < d.Ntot;
  const int r = in ? d.robot_of[g] : d.robot_of[d.Ntot - 1];
  const bool live = in && !d.st_done[r];
  double v = -1.0;
  if (live) {
    const int64_t o = d.off[r];
    const int64_t i = g - o;
    if (i == 0) {
      double dx0[3];
      base_increment(d, r, o, dx0);
      v = sqrt(dx0[0] * dx0[0] + dx0[1] * dx0[1] + dx0[2] * dx0[2]);
    } else {
      const double* z = d.Z + d.zoff[r] + 6 * (i - 1);
      v = sqrt(z[0] * z[0] + z[1] * z[1] + z[2] * z[2]);
      if (!(v >= 0.0)) v = -1.0;
    }
  }
  step_max(d, r, v);
}

// phase 4b of the exact method: the step dx = K^-1 (b + A^T y), with b the right-hand side that
// check_rhs_kernel wrote to Z's column 0 and y the forces of the active contacts, through the
// two-ended factor of phase 2, in place in Z's column 0, and each robot's largest node
// translation.  First every free node adds the forces of its active contacts to b (one thread
// per node; a contact along an element gives (1 - s) y n and s y n to its two nodes); then each side of a robot is a chain of dependent 6x6 block steps: forward from
// its end to the middle (base side f = 0 .. m-1, tip side f = nf-1 .. m+1), the middle node
// combines both, backward from the middle out.  A group of SSC lanes runs one chain: per chunk
// of SSN positions, one per lane, every lane turns its position's blocks into the step's affine
// map (forward y = c - G y_prev with G = L^-1 X, c = L^-1 b; backward x = c - H x_prev with
// H = L^-T X^T, c = L^-T y) and stages it in LDS; the group's first lane then runs the chain of
// 6x6 products while the group's loads of the next chunk are in flight.  Two robots per
// wavefront, neighbours in order of decreasing length.
__global__ void __launch_bounds__(256) add_forces_kernel(Dev d) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= d.Ntot) return;
  const int r = d.robot_of[g];
  if (d.st_done[r]) return;
  const int64_t o = d.off[r], i = g - o;
  const int nact = d.st_nact[r];
  if (i == 0 || nact == 0) return;
  const int64_t cb = (int64_t)r * d.cap;
  // the active contacts of node i (weight 1 - s) and along the element i-1 -> i (weight s);
  // the active list is in contact order, i.e. by node
  int lo = 0, hi = nact;               // first active contact at node >= i - 1
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (d.ct_node[cb + d.ac_idx[cb + mid]] < i - 1) lo = mid + 1; else hi = mid;
  }
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  bool any = false;
  for (int a = lo; a < nact; ++a) {
    const int64_t ci = cb + d.ac_idx[cb + a];
    const int64_t ic = d.ct_node[ci];
    if (ic > i) break;
    const double sv = d.ct_s[ci];
    if (ic < i && !(sv > 0.0)) continue;
    const double y = d.ac_y[cb + a] * (ic == i ? 1.0 - sv : sv);
    a0 += y * d.ct_n[3 * ci];
    a1 += y * d.ct_n[3 * ci + 1];
    a2 += y * d.ct_n[3 * ci + 2];
    any = true;
  }
  if (any) {
    double* z = d.Z + d.zoff[r] + 6 * (i - 1);
    z[0] += a0;
    z[1] += a1;
    z[2] += a2;
  }
}

constexpr int SSC = 16;                    // lanes per chain
constexpr int SSR = 64 / (2 * SSC);        // robots per wavefront
constexpr int SSN = SSC;                   // positions per staged chunk, one per lane
constexpr int SSG = 36 + 6;                // staged entries per position: G and c

__global__ void __launch_bounds__(64) step_solve_kernel(Dev d) {
  const int lane = threadIdx.x;
  const int g = lane / SSC, j = lane % SSC;   // chain g of the wavefront, lane j in its group
  const int k = blockIdx.x * SSR + g / 2;
  const bool tip = (g & 1) != 0;
  const int na = d.wl_cnt[WL_ACT];
  const int r = k < na ? d.wl[WL_ACT * d.B + k] : 0;   // neighbours in the list: similar lengths
  const bool live = k < na && !d.st_done[r];
  if (__ballot(live) == 0ull) return;
  const int64_t o = d.off[r], n = d.off[r + 1] - o, nf = n - 1, m = nf / 2;
  double* z = d.Z + d.zoff[r];
  const double* LD = d.LD + (o + 1) * 36;     // block of free node f at LD + 36 f
  const double* LS = d.LS + (o + 1) * 36;
  // this side's positions p = 0 .. cnt-1 from its end towards the middle, node f(p)
  const int64_t cnt = live ? (tip ? nf - 1 - m : m) : 0;
  const int64_t nch = (cnt + SSN - 1) / SSN;
  long long mc = nch;
#pragma unroll
  for (int sh = 32; sh > 0; sh >>= 1) mc = max(mc, (long long)__shfl_xor(mc, sh));
  const int64_t trips = mc;
  auto fnode = [&](int64_t p) { return tip ? nf - 1 - p : p; };
  __shared__ double sC[2 * SSR][SSN * SSG];
  double* C = sC[g];
  double px[36], pl[21], pv[6];
  // lane j of the group loads position ch * SSN + j of chunk ch (forward: p, backward: the
  // position cnt-1-p from the middle): the coupling X (forward: of the previous node, backward:
  // of the node), L's lower triangle by rows and the vector (forward: b, backward: y)
  auto fetch = [&](int64_t ch, bool fwd) {
    const int64_t pos = ch * SSN + j;
    const bool in = pos < cnt;
    const int64_t p = in ? (fwd ? pos : cnt - 1 - pos) : 0;
    const int64_t f = fnode(p);
    const int64_t xs = fwd ? (p >= 1 ? fnode(p - 1) : -1) : f;
    const bool hx = in && xs >= 0;
    const double* X = LS + 36 * (hx ? xs : 0);
    const double* L = LD + 36 * f;
#pragma unroll
    for (int q = 0; q < 36; ++q) px[q] = hx ? X[q] : 0.0;
#pragma unroll
    for (int a = 0, q = 0; a < 6; ++a)
#pragma unroll
      for (int b = 0; b <= a; ++b, ++q) pl[q] = in ? L[a * 6 + b] : 1.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) pv[q] = in ? z[6 * f + q] : 0.0;
  };
  auto Lr = [&](int a, int b) { return pl[a * (a + 1) / 2 + b]; };   // b <= a; diagonal: 1/L_aa
  // forward: G = L^-1 X and c = L^-1 b of the lane's position into LDS
  auto prep_fwd = [&]() {
#pragma unroll
    for (int b = 0; b < 6; ++b) {
      double col[6];
#pragma unroll
      for (int a = 0; a < 6; ++a) {
        double v = px[a * 6 + b];
#pragma unroll
        for (int q = 0; q < a; ++q) v -= Lr(a, q) * col[q];
        col[a] = v * Lr(a, a);
      }
#pragma unroll
      for (int a = 0; a < 6; ++a) C[j * SSG + a * 6 + b] = col[a];
    }
    double cv[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      double v = pv[a];
#pragma unroll
      for (int q = 0; q < a; ++q) v -= Lr(a, q) * cv[q];
      cv[a] = v * Lr(a, a);
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) C[j * SSG + 36 + a] = cv[a];
  };
  // backward: H = L^-T X^T and c = L^-T y of the lane's position into LDS
  auto prep_bwd = [&]() {
#pragma unroll
    for (int b = 0; b < 6; ++b) {
      double col[6];
#pragma unroll
      for (int a = 5; a >= 0; --a) {
        double v = px[b * 6 + a];                    // X^T (a, b)
#pragma unroll
        for (int q = a + 1; q < 6; ++q) v -= Lr(q, a) * col[q];
        col[a] = v * Lr(a, a);
      }
#pragma unroll
      for (int a = 0; a < 6; ++a) C[j * SSG + a * 6 + b] = col[a];
    }
    double cv[6];
#pragma unroll
    for (int a = 5; a >= 0; --a) {
      double v = pv[a];
#pragma unroll
      for (int q = a + 1; q < 6; ++q) v -= Lr(q, a) * cv[q];
      cv[a] = v * Lr(a, a);
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) C[j * SSG + 36 + a] = cv[a];
  };
  // the chain step v <- c - G v of staged position u
  auto chain = [&](int u, double (&v)[6]) {
    double nv[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      double s = C[u * SSG + 36 + a];
#pragma unroll
      for (int b = 0; b < 6; ++b) s -= C[u * SSG + a * 6 + b] * v[b];
      nv[a] = s;
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) v[a] = nv[a];
  };
  // ---------------------------------------------------------------- forward sweeps
  // y_p = L^-1 (b_p - X y_{p-1}) = c_p - G_p y_{p-1}
  double yp[6] = {0, 0, 0, 0, 0, 0};
  if (nch > 0) fetch(0, true);
  for (int64_t t = 0; t < trips; ++t) {
    __syncthreads();
    if (t < nch) prep_fwd();
    __syncthreads();
    if (t + 1 < nch) fetch(t + 1, true);
    if (j == 0 && t < nch) {
      for (int u = 0; u < SSN; ++u) {
        const int64_t p = t * SSN + u;
        if (p >= cnt) break;
        chain(u, yp);
        double* zf = z + 6 * fnode(p);
#pragma unroll
        for (int a = 0; a < 6; ++a) zf[a] = yp[a];
      }
    }
  }
  // ---------------------------------------------------------------- middle node
  const int base_lead = (g & ~1) * SSC, tip_lead = (g | 1) * SSC;
  double yt[6];                                       // the tip side's last forward value
#pragma unroll
  for (int a = 0; a < 6; ++a) yt[a] = __shfl(yp[a], tip_lead);
  double xm[6] = {0, 0, 0, 0, 0, 0};
  if (live && !tip && j == 0) {
    double bv[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) bv[a] = z[6 * m + a];
    const bool ht = m >= 1, hb = m + 1 < nf;
    const double* Xt = LS + 36 * (ht ? m - 1 : m);    // X_{m-1} (base side), if any
    const double* Xb = LS + 36 * (hb ? m + 1 : m);    // X_{m+1} (tip side), if any
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = 0; b < 6; ++b) {
        if (ht) bv[a] -= Xt[a * 6 + b] * yp[b];
        if (hb) bv[a] -= Xb[a * 6 + b] * yt[b];
      }
    const double* Lm = LD + 36 * m;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      const double y = bv[a] * Lm[a * 7];
      bv[a] = y;
#pragma unroll
      for (int b = a + 1; b < 6; ++b) bv[b] -= Lm[b * 6 + a] * y;
    }
#pragma unroll
    for (int a = 5; a >= 0; --a) {
      const double x = bv[a] * Lm[a * 7];
      xm[a] = x;
      z[6 * m + a] = x;
#pragma unroll
      for (int b = 0; b < a; ++b) bv[b] -= Lm[a * 6 + b] * x;
    }
  }
  double xn[6];
#pragma unroll
  for (int a = 0; a < 6; ++a) xn[a] = __shfl(xm[a], base_lead);
  // the largest translation: the base node's increment and the middle node (base side)
  double mx = -1.0;
  if (live && !tip && j == 0) {
    double dx0[3];
    base_increment(d, r, o, dx0);
    const double vb = sqrt(dx0[0] * dx0[0] + dx0[1] * dx0[1] + dx0[2] * dx0[2]);
    const double vm = sqrt(xn[0] * xn[0] + xn[1] * xn[1] + xn[2] * xn[2]);
    if (vb >= 0.0) mx = fmax(mx, vb);
    if (vm >= 0.0) mx = fmax(mx, vm);
  }
  __syncthreads();                                    // the forward values are in Z
  // ---------------------------------------------------------------- backward sweeps
  // position p = cnt-1-pos: x_f = L_f^-T (y_f - X_f^T x_neighbour) = c_f - H_f x_neighbour
  if (nch > 0) fetch(0, false);
  for (int64_t t = 0; t < trips; ++t) {
    __syncthreads();
    if (t < nch) prep_bwd();
    __syncthreads();
    if (t + 1 < nch) fetch(t + 1, false);
    if (j == 0 && t < nch) {
      for (int u = 0; u < SSN; ++u) {
        const int64_t pos = t * SSN + u;
        if (pos >= cnt) break;
        chain(u, xn);
        double* zf = z + 6 * fnode(cnt - 1 - pos);
#pragma unroll
        for (int a = 0; a < 6; ++a) zf[a] = xn[a];
        const double v = sqrt(xn[0] * xn[0] + xn[1] * xn[1] + xn[2] * xn[2]);
        if (v >= 0.0) mx = fmax(mx, v);
      }
    }
  }
  const double mt = __shfl(mx, tip_lead);
  if (live && !tip && j == 0) {
    const double v = fmax(mx, mt);
    d.st_mx[r] = v >= 0.0 ? (unsigned long long)__double_as_longlong(v) : 0ull;
  }
}

// phase 4c, one thread per node: the step-size limit (eq. 25-27: scale the step so that no
// node moves more than beta, beta halved every 10 contact-set switches) and the state
// update; the robot's contacts become the previous list (forces scaled with the step).
__global__ void __launch_bounds__(256) step_apply_kernel(Dev d) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= d.Ntot) return;
  const int r = d.robot_of[g];
  if (d.st_done[r]) return;
  const int64_t N = d.Ntot;
  const int64_t o = d.off[r], n = d.off[r + 1] - o;
  const int64_t i = g - o;
  const double mx = __longlong_as_double((long long)d.st_mx[r]);
  const int nsw = d.st_nswitch[r];
  const double beta = d.beta0 * fmax(1.0 / 64.0, ldexp(1.0, -(nsw / 10)));
  const bool limited = mx > beta;
  const double sc = limited ? beta / mx : 1.0;
  if (i == 0) {
    // base node: translation only
    double dx0[3];
    base_increment(d, r, o, dx0);
    for (int k = 0; k < 3; ++k) d.X[k * N + o] += sc * dx0[k];
  } else {
    const double* z = d.Z + d.zoff[r] + 6 * (i - 1);
    for (int k = 0; k < 3; ++k) d.X[k * N + g] += sc * z[k];
    const double wx = sc * z[3], wy = sc * z[4], wz = sc * z[5];
    const double th = sqrt(wx * wx + wy * wy + wz * wz);
    double cw, sw;
    if (th < 1e-8) {
      cw = 1.0 - th * th / 8.0;
      sw = 0.5 - th * th / 48.0;          // sin(th/2)/th
    } else {
      cw = cos(0.5 * th);
      sw = sin(0.5 * th) / th;
    }
    const double ew = cw, ex = sw * wx, ey = sw * wy, ez = sw * wz;
    const double qw = d.X[3 * N + g], qx = d.X[4 * N + g], qy = d.X[5 * N + g], qz = d.X[6 * N + g];
    double nw = ew * qw - ex * qx - ey * qy - ez * qz;
    double nx = ew * qx + ex * qw + ey * qz - ez * qy;
    double ny = ew * qy - ex * qz + ey * qw + ez * qx;
    double nz = ew * qz + ex * qy - ey * qx + ez * qw;
    const double inv = 1.0 / sqrt(nw * nw + nx * nx + ny * ny + nz * nz);
    d.X[3 * N + g] = nw * inv; d.X[4 * N + g] = nx * inv; d.X[5 * N + g] = ny * inv; d.X[6 * N + g] = nz * inv;
  }
  const int nc = d.st_nc[r];
  const int64_t cb = (int64_t)r * d.cap;
  for (int64_t c = i; c < nc; c += n) {
    d.cp_node[cb + c] = d.ct_node[cb + c];
    d.cp_tri[cb + c] = d.ct_tri[cb + c];
    d.cp_kind[cb + c] = d.ct_kind[cb + c];
    d.cp_gap[cb + c] = d.ct_gap[cb + c];
    d.cp_y[cb + c] = sc * d.ct_y[cb + c];
    d.cp_s[cb + c] = d.ct_s[cb + c];
    for (int k = 0; k < 3; ++k) d.cp_n[3 * (cb + c) + k] = d.ct_n[3 * (cb + c) + k];
  }
  if (i == 0) {
    d.st_ncp[r] = nc;
    d.st_limited[r] = limited ? 1 : 0;
    d.st_nlim[r] += limited ? 1 : 0;
    const int it = d.st_it[r];
    d.st_iters[r] = it + 1;
    d.st_it[r] = it + 1;
  }
}

// phase 4 for robots with at most LCPM contacts: W packed in LDS, the wavefront LCP
__global__ void __launch_bounds__(NT) update_kernel(Dev d) {
  if ((int)blockIdx.x >= d.wl_cnt[WL_SMALL]) return;
  const int r = d.wl[WL_SMALL * d.B + blockIdx.x];   // longest robots first
  const int lane = threadIdx.x;
  if (d.st_done[r]) return;
  const int nc = d.st_nc[r];
  if (nc > LCPM) return;               // update_wide_kernel
  const int64_t cb = (int64_t)r * d.cap;
  const double* Wr = d.W + cb * d.zp;
  __shared__ LcpLds S;
  __shared__ int s_lcp_ok;
  double* qv = d.q + cb;
  double* y = d.ct_y + cb;
  contact_q(d, cb, nc, Wr, qv);
  // W packed in LDS: lane a takes its row of products, W(a, b) = n_a . Z_b(node of a), b <= a
  bool warm = false;
  if (lane < nc) {
    const double* wa = Wr + (int64_t)lane * d.zp + 1;
#pragma unroll 8
    for (int b = 0; b <= lane; ++b) S.W[pk(lane, b)] = wa[b];
    warm = d.ct_warm[cb + lane] != 0;
  }
  __syncthreads();
  double yl = 0.0;
  bool ok = true;
  if (nc > 0) ok = lcp_parallel(S, qv, nc, warm, yl);
  if (lane < nc) y[lane] = yl;
  if (lane == 0) s_lcp_ok = ok ? 1 : 0;
  __syncthreads();
  if (!s_lcp_ok) {
    finish(d, r, 2, d.st_it[r], d.st_rn[r]);
    return;
  }
  store_active(d, r, nc);
}

// ---------------------------------------------------------------- wide LCP (nc > LCPM)
// The same primal active-set method for contact sets beyond LCPM, one wavefront per robot.
// Constraint i is handled by lane i % NT; active position p by lane p % NT (SP per lane).
// W is read by columns (column t at Wc + t * ld; for a robot's contact set the rows of
// contact products that the substitution wrote, W being symmetric).  The Cholesky factor of the active block, packed with rows in
// order of entry, lives in LDS up to NPW positions; a set that outgrows it is solved again
// with the factor in device memory (up to every constraint).
constexpr int NPW = 128;
constexpr int CAPW = 1024;             // largest contact capacity (host-checked)
constexpr int SPL = NPW / NT;          // positions per lane, factor in LDS
constexpr int SPG = CAPW / NT;         // positions per lane, factor in device memory

struct LcpWideLds {
  double L[NPW * (NPW + 1) / 2];
  double Rd[NPW];
  double Yp[NPW];
  int P[NPW];
  double Q[CAPW];                      // q by constraint
  unsigned char In[CAPW];              // constraint i is in the active set
  unsigned char Wm[CAPW];              // constraint i starts in the active set (warm start)
};

// where the factor of the active block lives: packed lower L (true off-diagonal entries),
// reciprocal diagonal Rd, active y and constraint index by position, capacity npmax
struct LcpWs {
  double* L;
  double* Rd;
  double* Yp;
  int* P;
  int npmax;
};

// the contact products of a robot's contact set, formed by the substitution: "column" t is
// read as the contiguous row of contact t, W(t, i) = n_t . Z_i(node of t), which equals
// W(i, t) (W is symmetric) up to rounding; warm-start flags from the contact list
struct RobotLcpSource {
  const decltype(Dev::ct_warm) wf;     // the robot's warm-start flags
  __device__ bool warm(int i) const { return wf[i] != 0; }
};

// a given dense W (column-major, ld = cap), no warm start
struct DenseLcpSource {
  __device__ bool warm(int) const { return false; }
};

template <int SP>
__device__ __forceinline__ double wide_pick(const double (&v)[SP], int s) {
  double x = v[0];
#pragma unroll
  for (int u = 1; u < SP; ++u)
    if (s == u) x = v[u];
  return x;
}

// L x = b over positions < np, in place (b, x by position)
template <int SP>
__device__ __forceinline__ void wide_fwd(const LcpWs& w, int np, double (&bv)[SP]) {
  const int lane = threadIdx.x;
  if (np <= NT) {                      // one position per lane
    bv[0] = tri_fwd1(w.L, w.Rd, np, bv[0]);
    return;
  }
  for (int k = 0; k < np; ++k) {
    const double xk = lane_read(wide_pick<SP>(bv, k / NT), k % NT) * w.Rd[k];
#pragma unroll
    for (int s = 0; s < SP; ++s) {
      if (s * NT >= np) break;
      if ((s + 1) * NT <= k) continue;
      const int p = lane + NT * s;
      if (p == k) bv[s] = xk;
      else if (p > k && p < np) bv[s] -= w.L[pk(p, k)] * xk;
    }
  }
}

// L^T x = b over positions < np, in place
template <int SP>
__device__ __forceinline__ void wide_bwd(const LcpWs& w, int np, double (&bv)[SP]) {
  const int lane = threadIdx.x;
  if (np <= NT) {
    bv[0] = tri_bwd1(w.L, w.Rd, np, bv[0]);
    return;
  }
  for (int k = np - 1; k >= 0; --k) {
    const double xk = lane_read(wide_pick<SP>(bv, k / NT), k % NT) * w.Rd[k];
#pragma unroll
    for (int s = 0; s < SP; ++s) {
      if (s * NT > k) break;
      const int p = lane + NT * s;
      if (p == k) bv[s] = xk;
      else if (p < k) bv[s] -= w.L[pk(k, p)] * xk;
    }
  }
}

// Cholesky of W(P, P) over np positions, by columns (position p on lane p % NT): up to NT
// positions by chol_cols1, beyond that with the sums of a column formed directly
template <int SP>
__device__ bool wide_factor(const LcpWs& w, const double* Wc, int cap, int np) {
  const int lane = threadIdx.x;
  // W(P, P) into the packed rows: the constraint indices by lane reads, eight loads in flight
  // per lane before their writes
  int pr[SP];
#pragma unroll
  for (int s = 0; s < SP; ++s) pr[s] = lane + NT * s < np ? w.P[lane + NT * s] : 0;
#pragma unroll
  for (int s = 0; s < SP; ++s) {
    if (s * NT >= np) break;
    const int p = lane + NT * s;
    const int bend = np < (s + 1) * NT ? np : (s + 1) * NT;   // b <= p < bend
    for (int b0 = 0; b0 < bend; b0 += 8) {
      double v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int b = b0 + e < bend ? b0 + e : 0;
        int pb = pr[0];
#pragma unroll
        for (int u = 1; u < SP; ++u)
          if (b / NT == u) pb = pr[u];
        pb = __builtin_amdgcn_readlane(pb, b % NT);
        v[e] = p < np && b0 + e <= p ? Wc[(int64_t)pb * cap + pr[s]] : 0.0;
      }
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (p < np && b0 + e <= p) w.L[pk(p, b0 + e)] = v[e];
    }
  }
  __syncthreads();
  if (np <= NT) return chol_cols1(w.L, w.Rd, np);
  bool ok = true;
  for (int j = 0; j < np; ++j) {
    const double* Lj = w.L + pk(j, 0);
    double a[SP];
#pragma unroll
    for (int s = 0; s < SP; ++s) a[s] = 0.0;
#pragma unroll
    for (int s = 0; s < SP; ++s) {
      if (s * NT >= np) break;
      if ((s + 1) * NT <= j) continue;
      const int p = lane + NT * s;
      if (p >= j && p < np) {
        const double* Lp = w.L + pk(p, 0);
        double v = Lp[j];
#pragma unroll 8
        for (int k = 0; k < j; ++k) v -= Lp[k] * Lj[k];
        a[s] = v;
      }
    }
    const double piv = lane_read(wide_pick<SP>(a, j / NT), j % NT);
    if (!(piv > 0.0)) ok = false;
    const double rk = rsqrt_nr(piv > 0.0 ? piv : 1.0);
#pragma unroll
    for (int s = 0; s < SP; ++s) {
      if (s * NT >= np) break;
      if ((s + 1) * NT <= j) continue;
      const int p = lane + NT * s;
      if (p >= j && p < np) w.L[pk(p, j)] = p == j ? a[s] : a[s] * rk;
    }
    if (lane == 0) w.Rd[j] = rk;
    __syncthreads();
  }
  return ok;
}

// 0: solved (y written), 1: non-positive pivot or iteration limit, 2: active set beyond npmax.
template <int SP, class Src>
__device__ int lcp_wide(const Src& src, LcpWideLds& S, const LcpWs& w, const double* Wc, int cap,
                        const double* q, int m, double* y) {
  const int lane = threadIdx.x;
  // q and the warm-start flags staged in LDS (their loads in flight together)
  double qmax = 0.0;
#pragma unroll 4
  for (int i = lane; i < m; i += NT) {
    const double qq = q[i];
    const bool wf = src.warm(i);
    qmax = fmax(qmax, fabs(qq));
    S.Q[i] = qq;
    S.In[i] = 0;
    S.Wm[i] = wf ? 1 : 0;
  }
  const double tolw = 1e-12 * warp_max(qmax);
  __syncthreads();
  int np = 0;
  // warm start from the constraints the source flags (previous iterate's active contacts)
  {
    int cnt = 0;
    for (int i0 = 0; i0 < m; i0 += NT) {
      const int i = i0 + lane;
      const bool wf = i < m && S.Wm[i] != 0;
      const unsigned long long wm = __ballot(wf);
      const int pos = cnt + __popcll(wm & ((1ull << lane) - 1ull));
      if (wf && pos < w.npmax) w.P[pos] = i;
      cnt += __popcll(wm);
    }
    __syncthreads();
    if (cnt > w.npmax) cnt = 0;
    // solve on the set, drop the constraints whose y is not positive, solve again
    while (cnt > 0) {
      if (!wide_factor<SP>(w, Wc, cap, cnt)) break;
      double z[SP];
#pragma unroll
      for (int s = 0; s < SP; ++s) {
        const int p = lane + NT * s;
        z[s] = p < cnt ? -S.Q[w.P[p]] : 0.0;
      }
      wide_fwd<SP>(w, cnt, z);
      wide_bwd<SP>(w, cnt, z);
      bool bad = false;
#pragma unroll
      for (int s = 0; s < SP; ++s) bad |= (lane + NT * s < cnt) && !(z[s] > 0.0);
      if (__ballot(bad) == 0ull) {
#pragma unroll
        for (int s = 0; s < SP; ++s) {
          const int p = lane + NT * s;
          if (p < cnt) { w.Yp[p] = z[s]; S.In[w.P[p]] = 1; }
        }
        np = cnt;
        __syncthreads();
        break;
      }
      int pidx[SP];
      unsigned long long km[SP];
#pragma unroll
      for (int s = 0; s < SP; ++s) {
        const int p = lane + NT * s;
        pidx[s] = p < cnt ? w.P[p] : 0;
        km[s] = __ballot(p < cnt && z[s] > 0.0);
      }
      __syncthreads();
      int base = 0;
#pragma unroll
      for (int s = 0; s < SP; ++s) {
        if ((km[s] >> (threadIdx.x & 63)) & 1ull) w.P[base + __popcll(km[s] & ((1ull << lane) - 1ull))] = pidx[s];
        base += __popcll(km[s]);
      }
      cnt = base;
      __syncthreads();
    }
  }
  bool done = false, failed = false, full = false;
  for (int outer = 0; outer < 4 * m + 8 && !done && !failed; ++outer) {
    // most violated inactive constraint: w_i = q_i + sum_a W(i, P_a) y_a
    double v = INFINITY;
    int t = 0x7fffffff;
    for (int i0 = 0; i0 < m; i0 += 4 * NT) {   // 4 constraints per lane, loads in flight together
      double wv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + lane + u * NT;
        wv[u] = i < m ? S.Q[i] : 0.0;
      }
      // eight columns at a time, the last group masked: their 32 loads are in flight together
      // (accumulation in column order)
      for (int a = 0; a < np; a += 8) {
        double ya[8], cv[8][4];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const bool ce = a + e < np;
          ya[e] = ce ? w.Yp[a + e] : 0.0;
          const double* col = Wc + (int64_t)(ce ? w.P[a + e] : 0) * cap;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int i = i0 + lane + u * NT;
            cv[e][u] = ce && i < m ? col[i] : 0.0;
          }
        }
#pragma unroll
        for (int e = 0; e < 8; ++e)
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (a + e < np && i0 + lane + u * NT < m) wv[u] += cv[e][u] * ya[e];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + lane + u * NT;
        if (i < m && !S.In[i] && wv[u] < -tolw && wv[u] < v) { v = wv[u]; t = i; }
      }
    }
    wave_argmin(v, t);
    if (!(v < INFINITY)) { done = true; break; }
    if (np == w.npmax) { full = true; break; }
    // append t: the new factor row l solves L l = W(P, t)
    double bv[SP];
#pragma unroll
    for (int s = 0; s < SP; ++s) {
      const int p = lane + NT * s;
      bv[s] = p < np ? Wc[(int64_t)t * cap + w.P[p]] : 0.0;
    }
    wide_fwd<SP>(w, np, bv);
    double ss = 0.0;
#pragma unroll
    for (int s = 0; s < SP; ++s) ss += (lane + NT * s < np) ? bv[s] * bv[s] : 0.0;
    const double dtt = Wc[(int64_t)t * cap + t] - warp_sum(ss);
    __syncthreads();
    if (dtt > 0.0) {
#pragma unroll
      for (int s = 0; s < SP; ++s) {
        const int p = lane + NT * s;
        if (p < np) w.L[pk(np, p)] = bv[s];
      }
      if (lane == 0) {
        w.L[pk(np, np)] = 1.0;
        w.Rd[np] = rsqrt_nr(dtt);
        w.P[np] = t;
        w.Yp[np] = 0.0;
        S.In[t] = 1;
      }
      ++np;
      __syncthreads();
    } else {
      // t depends linearly on the active set: exchange it for the first active constraint
      // whose y reaches zero along y_P - s c, c = W_PP^-1 W(P, t) (every w unchanged)
      wide_bwd<SP>(w, np, bv);
      double cmax = 0.0;
#pragma unroll
      for (int s = 0; s < SP; ++s) cmax = fmax(cmax, (lane + NT * s < np) ? fabs(bv[s]) : 0.0);
      cmax = warp_max(cmax);
      double rat = INFINITY;
      int jp = 0x7fffffff;
#pragma unroll
      for (int s = 0; s < SP; ++s) {
        const int p = lane + NT * s;
        if (p < np && bv[s] > 1e-12 * cmax) {
          const double r = w.Yp[p] / bv[s];
          if (r < rat) { rat = r; jp = p; }
        }
      }
      wave_argmin(rat, jp);
      if (!(rat < INFINITY)) { failed = true; break; }
      double yv[SP];
#pragma unroll
      for (int s = 0; s < SP; ++s) {
        const int p = lane + NT * s;
        yv[s] = p < np ? (p == jp ? rat : fmax(w.Yp[p] - rat * bv[s], 0.0)) : 0.0;
      }
      const int oldj = w.P[jp];
      __syncthreads();
#pragma unroll
      for (int s = 0; s < SP; ++s) {
        const int p = lane + NT * s;
        if (p < np) w.Yp[p] = yv[s];
      }
      if (lane == 0) { S.In[oldj] = 0; w.P[jp] = t; S.In[t] = 1; }
      __syncthreads();
      if (!wide_factor<SP>(w, Wc, cap, np)) { failed = true; break; }
    }
    for (int inner = 0; inner < 4 * m + 8; ++inner) {
      double z[SP];
#pragma unroll
      for (int s = 0; s < SP; ++s) {
        const int p = lane + NT * s;
        z[s] = p < np ? -S.Q[w.P[p]] : 0.0;
      }
      wide_fwd<SP>(w, np, z);
      wide_bwd<SP>(w, np, z);
      bool bad = false;
#pragma unroll
      for (int s = 0; s < SP; ++s) bad |= (lane + NT * s < np) && !(z[s] > 0.0);
      if (__ballot(bad) == 0ull) {
#pragma unroll
        for (int s = 0; s < SP; ++s) {
          const int p = lane + NT * s;
          if (p < np) w.Yp[p] = z[s];
        }
        __syncthreads();
        break;
      }
      // step toward z until the first active y reaches zero
      double al = 1.0;
#pragma unroll
      for (int s = 0; s < SP; ++s) {
        const int p = lane + NT * s;
        if (p < np && z[s] <= 0.0) {
          const double yp = w.Yp[p];
          al = fmin(al, yp / (yp - z[s]));
        }
      }
      al = fmin(1.0, warp_min(al));
      double yn[SP];
      int pidx[SP];
      unsigned long long km[SP];
#pragma unroll
      for (int s = 0; s < SP; ++s) {
        const int p = lane + NT * s;
        const double yp = p < np ? w.Yp[p] : 0.0;
        yn[s] = yp + al * (z[s] - yp);
        pidx[s] = p < np ? w.P[p] : 0;
        km[s] = __ballot(p < np && yn[s] > 0.0);
      }
      __syncthreads();
      int base = 0;
#pragma unroll
      for (int s = 0; s < SP; ++s) {
        const int p = lane + NT * s;
        const bool keep = p < np && yn[s] > 0.0;
        if (p < np && !keep) S.In[pidx[s]] = 0;
        if (keep) {
          const int pos = base + __popcll(km[s] & ((1ull << lane) - 1ull));
          w.P[pos] = pidx[s];
          w.Yp[pos] = yn[s];
        }
        base += __popcll(km[s]);
      }
      np = base;
      __syncthreads();
      if (np == 0) break;
      if (!wide_factor<SP>(w, Wc, cap, np)) { failed = true; break; }
    }
  }
  if (full) return 2;
  if (failed || !done) return 1;
  for (int i = lane; i < m; i += NT) y[i] = 0.0;
  __syncthreads();
#pragma unroll
  for (int s = 0; s < SP; ++s) {
    const int p = lane + NT * s;
    if (p < np) y[w.P[p]] = w.Yp[p];
  }
  __syncthreads();
  return 0;
}

// the factor workspace in device memory for m constraints: packed L, Rd, Yp, P
__device__ __forceinline__ LcpWs global_ws(double* g, int m) {
  const int64_t nl = (int64_t)m * (m + 1) / 2;
  return LcpWs{g, g + nl, g + nl + m, (int*)(g + nl + 2 * m), m};
}

// phase 4 for robots with more than LCPM contacts
__global__ void __launch_bounds__(NT) update_wide_kernel(Dev d) {
  if ((int)blockIdx.x >= d.wl_cnt[WL_WIDE]) return;
  const int r = d.wl[WL_WIDE * d.B + blockIdx.x];   // longest robots first
  if (d.st_done[r]) return;
  const int nc = d.st_nc[r];
  if (nc <= LCPM) return;              // update_kernel
  const int64_t cb = (int64_t)r * d.cap;
  __shared__ LcpWideLds S;
  double* qv = d.q + cb;
  double* y = d.ct_y + cb;
  double* Wr = d.W + cb * d.zp;
  contact_q(d, cb, nc, Wr, qv);
  __syncthreads();
  const RobotLcpSource src{d.ct_warm + cb};
  const LcpWs wl{S.L, S.Rd, S.Yp, S.P, NPW};
  const int code = lcp_wide<SPL>(src, S, wl, Wr + 1, (int)d.zp, qv, nc, y);
  if (threadIdx.x == 0 && code == 2) d.wl[WL_BIG * d.B + atomicAdd(&d.wl_cnt[WL_BIG], 1)] = r;
  if (code == 1) {
    finish(d, r, 2, d.st_it[r], d.st_rn[r]);
    return;
  }
  if (code == 0) store_active(d, r, nc);
}

// phase 4 for the robots whose wide LCP outgrew the LDS factor: the same method again with the
// factor in the robot's device workspace (up to every constraint).  A kernel of its own, so
// that the common path keeps its registers (this one holds 16 positions per lane).
__global__ void __launch_bounds__(NT) update_big_kernel(Dev d) {
  if ((int)blockIdx.x >= d.wl_cnt[WL_BIG]) return;
  const int r = d.wl[WL_BIG * d.B + blockIdx.x];
  if (d.st_done[r]) return;
  const int nc = d.st_nc[r];
  if (nc <= LCPM) return;
  const int64_t cb = (int64_t)r * d.cap;
  __shared__ LcpWideLds S;
  const double* qv = d.q + cb;                  // written by update_wide_kernel
  double* y = d.ct_y + cb;
  double* Wr = d.W + cb * d.zp;
  const RobotLcpSource src{d.ct_warm + cb};
  if (lcp_wide<SPG>(src, S, global_ws(lcp_ws(d, r), nc), Wr + 1, (int)d.zp, qv, nc, y) != 0) {
    finish(d, r, 2, d.st_it[r], d.st_rn[r]);
    return;
  }
  store_active(d, r, nc);
}

// fem_lcp: the LCP routines above on a given W (column-major, ld = m), one block
__global__ void __launch_bounds__(NT) lcp_small_kernel(const double* W, const double* q, int m,
                                                       double* y, int* code) {
  __shared__ LcpLds S;
  const int lane = threadIdx.x;
  if (lane < m)
    for (int b = 0; b <= lane; ++b) S.W[pk(lane, b)] = W[(int64_t)b * m + lane];
  __syncthreads();
  double yl = 0.0;
  const bool ok = lcp_parallel(S, q, m, false, yl);
  if (lane < m) y[lane] = yl;
  if (lane == 0) *code = ok ? 0 : -1;
}

__global__ void __launch_bounds__(NT) lcp_wide_check_kernel(double* W, const double* q, int m,
                                                            double* y, int* code) {
  __shared__ LcpWideLds S;
  const LcpWs wl{S.L, S.Rd, S.Yp, S.P, NPW};
  const int c = lcp_wide<SPL>(DenseLcpSource{}, S, wl, W, m, q, m, y);
  if (threadIdx.x == 0) *code = c == 0 ? 1 : (c == 2 ? 2 : -1);
}

// the set outgrew the LDS factor (code 2): again with the factor in device memory
__global__ void __launch_bounds__(NT) lcp_big_check_kernel(double* W, const double* q, int m,
                                                           double* y, double* gws, int* code) {
  if (*code != 2) return;
  __shared__ LcpWideLds S;
  const int c = lcp_wide<SPG>(DenseLcpSource{}, S, global_ws(gws, m), W, m, q, m, y);
  __syncthreads();
  if (threadIdx.x == 0) *code = c == 0 ? 2 : -1;
}

void launch_lcp_check(double* W, const double* q, int m, double* y, double* scratch, int* code,
                      hipStream_t s) {
  if (m <= LCPM) hipLaunchKernelGGL(lcp_small_kernel, dim3(1), dim3(NT), 0, s, W, q, m, y, code);
  else {
    hipLaunchKernelGGL(lcp_wide_check_kernel, dim3(1), dim3(NT), 0, s, W, q, m, y, code);
    hipLaunchKernelGGL(lcp_big_check_kernel, dim3(1), dim3(NT), 0, s, W, q, m, y, scratch, code);
  }
}

// detection-only path: compact the per-node contacts of every robot (no step)
__global__ void __launch_bounds__(NT) gather_kernel(Dev d) {
  const int r = blockIdx.x;
  int nc;
  bool ovf;
  gather_contacts(d, r, &nc, &ovf);
  __syncthreads();
  const int cap = d.cap;
  const int64_t cb = (int64_t)r * cap;
  if (!ovf) {
    for (int c = threadIdx.x; c < nc; c += NT) {
      d.cp_node[cb + c] = d.ct_node[cb + c];
      d.cp_tri[cb + c] = d.ct_tri[cb + c];
      d.cp_kind[cb + c] = d.ct_kind[cb + c];
      d.cp_gap[cb + c] = d.ct_gap[cb + c];
      d.cp_y[cb + c] = 0.0;
      d.cp_s[cb + c] = d.ct_s[cb + c];
      for (int k = 0; k < 3; ++k) d.cp_n[3 * (cb + c) + k] = d.ct_n[3 * (cb + c) + k];
    }
  }
  if (threadIdx.x == 0) {
    d.st_ncp[r] = ovf ? 0 : nc;
    d.st_nc[r] = nc;
  }
}

// ------------------------------------------------------------------ ADMM variant
// The QP of eq. 23 solved by the operator-splitting iteration of OSQP (the solver Sec. III-B
// uses; Stellato et al. 2020, Algorithm 1, without problem scaling, fixed penalty rho) instead
// of the exact Schur complement + LCP.  The QP over the free DOFs is
//     min 1/2 x^T K x - b^T x   subject to   A x + g >= 0
// (b = column 0 of Z as written by check_rhs_kernel: minus the out-of-balance force with the
// base coupling and prescribed increments moved over, prescribed DOFs as identity rows), and
// OSQP's multiplier y_o of l <= A x with l = -g is minus the contact force.  Per iteration
//     (K + sigma I + rho A^T A) xt = sigma x + b + A^T (rho z - y_o)
//     x <- alpha xt + (1 - alpha) x,  zr = alpha A xt + (1 - alpha) z
//     z <- max(zr + y_o / rho, -g),   y_o <- y_o + rho (zr - z)
// until |A x - z| and |K x - b + A^T y_o| (infinity norms over free DOFs) are below
// eps (1 + the scale OSQP uses).  Every contact row lies on one node, so K + sigma I +
// rho A^T A stays block tridiagonal: it is factored once per Newton iteration (one-ended
// block Cholesky, 6x6 blocks) and each iteration is one forward and one backward sweep.
// One wavefront per robot: the factorisation and the sweeps run serially in lane 0 (the
// variant exists for comparison with the exact method, which parallelises over the
// right-hand sides), the contact updates over lanes.  The result x goes to Z's column 0
// and the forces to the contact list, so the step kernels apply it like an exact step.
constexpr double ADMM_SIGMA = 1e-6, ADMM_ALPHA = 1.6;

// the node's 6x6 block of M = K + sigma I + rho A^T A, prescribed rows and columns -> identity
__device__ void admm_diag_block(const Dev& d, int r, int64_t o, int64_t n, int64_t i, const Guide& G,
                                int c0, int c1, int64_t cb, double* A) {
  const bool right = i < n - 1;
  const ElemK KL = load_elem(d, o + i - 1), KR = load_elem(d, o + (right ? i : i - 1));
  for (int a = 0; a < 6; ++a)
    for (int b = 0; b < 6; ++b) A[a * 6 + b] = k_bb(KL, a, b) + (right ? k_aa(KR, a, b) : 0.0);
  for (int a = 0; a < 6; ++a) A[a * 7] += ADMM_SIGMA;
  for (int c = c0; c < c1; ++c) {
    const double* nc = d.ct_n + 3 * (cb + c);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) A[a * 6 + b] += d.admm_rho * nc[a] * nc[b];
  }
  for (int a = 0; a < 6; ++a)
    for (int b = 0; b < 6; ++b)
      if (G.dof(i, a) || G.dof(i, b)) A[a * 6 + b] = (a == b) ? 1.0 : 0.0;
}

__global__ void __launch_bounds__(NT) admm_kernel(Dev d) {
  const int r = d.solve_order[blockIdx.x];   // longest robots first
  const int lane = threadIdx.x;
  if (d.st_done[r]) return;
  const int64_t o = d.off[r], n = d.off[r + 1] - o, nf = n - 1;
  const Guide G = make_guide(d, r, n);
  const int nc = d.st_nc[r];
  const int cap = d.cap;
  const int64_t cb = (int64_t)r * cap;
  const int64_t zp = d.zp;
  double* Yr = d.Y + 6 * o * zp;                 // per free DOF row: x, xt, v, K x in columns 0..3
  double* b0 = d.Z + d.zoff[r];                  // b (free DOF rows), then the result x
  double* ws = lcp_ws(d, r);
  double* zc = ws;                               // z, y_o per contact
  double* yo = ws + cap;
  const double rho = d.admm_rho, eps = d.admm_eps;
  __shared__ int s_fail, s_stop;
  if (lane == 0) { s_fail = 0; s_stop = 0; }
  // ---------------------------------------------------------------- factorisation (lane 0)
  if (lane == 0) {
    double Xp[36];
    for (int k = 0; k < 36; ++k) Xp[k] = 0.0;
    int cp = 0;
    for (int64_t f = 0; f < nf; ++f) {
      const int64_t i = f + 1, g = o + i;
      while (cp < nc && d.ct_node[cb + cp] < i) ++cp;
      int c1 = cp;
      while (c1 < nc && d.ct_node[cb + c1] == i) ++c1;
      double A[36];
      admm_diag_block(d, r, o, n, i, G, cp, c1, cb, A);
      cp = c1;
      for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) {
          double s = 0.0;
          for (int q = 0; q < 6; ++q) s += Xp[a * 6 + q] * Xp[b * 6 + q];
          A[a * 6 + b] -= s;
        }
      // lower Cholesky in place, reciprocal diagonal
      for (int q = 0; q < 6; ++q) {
        double dq = A[q * 7];
        for (int t = 0; t < q; ++t) dq -= A[q * 6 + t] * A[q * 6 + t];
        if (!(dq > 0.0)) { s_fail = 1; dq = 1.0; }
        const double rq = 1.0 / sqrt(dq);
        A[q * 7] = rq;
        for (int p = q + 1; p < 6; ++p) {
          double v = A[p * 6 + q];
          for (int t = 0; t < q; ++t) v -= A[p * 6 + t] * A[q * 6 + t];
          A[p * 6 + q] = v * rq;
        }
      }
      for (int k = 0; k < 36; ++k) d.LD[g * 36 + k] = A[k];
      // X = L_{i+1,i}: row a solves L x = C[:, a], C = K[i, i+1] without prescribed rows/columns
      double X[36];
      if (i < n - 1) {
        const ElemK KR = load_elem(d, o + i);
        for (int a = 0; a < 6; ++a) {
          double x[6];
          for (int q = 0; q < 6; ++q) {
            double v = (G.dof(i, q) || G.dof(i + 1, a)) ? 0.0 : k_ab(KR, q, a);
            for (int t = 0; t < q; ++t) v -= A[q * 6 + t] * x[t];
            x[q] = v * A[q * 7];
          }
          for (int q = 0; q < 6; ++q) X[a * 6 + q] = x[q];
        }
      } else {
        for (int k = 0; k < 36; ++k) X[k] = 0.0;
      }
      for (int k = 0; k < 36; ++k) { d.LS[g * 36 + k] = X[k]; Xp[k] = X[k]; }
    }
  }
  for (int64_t k = lane; k < 6 * nf; k += NT) {
    const int64_t f = k / 6;
    const int q = (int)(k % 6);
    Yr[k * zp + 0] = G.dof(f + 1, q) ? b0[k] : 0.0;   // x: prescribed rows at their increments
  }
  for (int c = lane; c < nc; c += NT) { zc[c] = 0.0; yo[c] = 0.0; }
  __syncthreads();
  if (s_fail) {
    finish(d, r, 3, d.st_it[r], d.st_rn[r]);
    return;
  }
  int it = 0;
  for (; it < d.admm_max_iter; ++it) {
    // ------------------------------------------------ x-update: one solve with M (lane 0)
    if (lane == 0) {
      double vp[6] = {0, 0, 0, 0, 0, 0};
      int cp = 0;
      for (int64_t f = 0; f < nf; ++f) {
        const int64_t i = f + 1, g = o + i;
        double v[6];
        for (int q = 0; q < 6; ++q) {
          const int64_t row = 6 * f + q;
          v[q] = G.dof(i, q) ? b0[row] : ADMM_SIGMA * Yr[row * zp] + b0[row];
        }
        while (cp < nc && d.ct_node[cb + cp] < i) ++cp;
        for (; cp < nc && d.ct_node[cb + cp] == i; ++cp) {
          const double w = rho * zc[cp] - yo[cp];
          for (int a = 0; a < 3; ++a)
            if (!G.dof(i, a)) v[a] += w * d.ct_n[3 * (cb + cp) + a];
        }
        if (f > 0) {
          const double* Xl = d.LS + (g - 1) * 36;     // L_{i,i-1}
          for (int p = 0; p < 6; ++p)
            for (int q = 0; q < 6; ++q) v[p] -= Xl[p * 6 + q] * vp[q];
        }
        const double* L = d.LD + g * 36;
        for (int q = 0; q < 6; ++q) {
          double s = v[q];
          for (int t = 0; t < q; ++t) s -= L[q * 6 + t] * vp[t];
          vp[q] = s * L[q * 7];
        }
        for (int q = 0; q < 6; ++q) Yr[(6 * f + q) * zp + 2] = vp[q];
      }
      double xn[6] = {0, 0, 0, 0, 0, 0};
      for (int64_t f = nf - 1; f >= 0; --f) {
        const int64_t i = f + 1, g = o + i;
        double v[6];
        for (int q = 0; q < 6; ++q) v[q] = Yr[(6 * f + q) * zp + 2];
        if (f < nf - 1) {
          const double* X = d.LS + g * 36;           // L_{i+1,i}
          for (int q = 0; q < 6; ++q)
            for (int p = 0; p < 6; ++p) v[q] -= X[p * 6 + q] * xn[p];
        }
        const double* L = d.LD + g * 36;
        double x[6];
        for (int q = 5; q >= 0; --q) {
          double s = v[q];
          for (int t = q + 1; t < 6; ++t) s -= L[t * 6 + q] * x[t];
          x[q] = s * L[q * 7];
        }
        for (int q = 0; q < 6; ++q) {
          xn[q] = x[q];
          const int64_t row = 6 * f + q;
          Yr[row * zp + 1] = x[q];
          Yr[row * zp + 0] = ADMM_ALPHA * x[q] + (1.0 - ADMM_ALPHA) * Yr[row * zp + 0];
        }
      }
    }
    __syncthreads();
    // ------------------------------------------------ z and y_o updates (lanes over contacts)
    double rp = 0.0, sAx = 0.0, sz = 0.0;
    for (int c = lane; c < nc; c += NT) {
      const int64_t f = d.ct_node[cb + c] - 1;
      const double* nv = d.ct_n + 3 * (cb + c);
      double zt = 0.0, ax = 0.0;
      for (int a = 0; a < 3; ++a) {
        zt += nv[a] * Yr[(6 * f + a) * zp + 1];
        ax += nv[a] * Yr[(6 * f + a) * zp + 0];
      }
      const double zr = ADMM_ALPHA * zt + (1.0 - ADMM_ALPHA) * zc[c];
      const double zn = fmax(zr + yo[c] / rho, -d.ct_gap[cb + c]);
      yo[c] += rho * (zr - zn);
      zc[c] = zn;
      rp = fmax(rp, fabs(ax - zn));
      sAx = fmax(sAx, fabs(ax));
      sz = fmax(sz, fabs(zn));
    }
    rp = warp_max(rp); sAx = warp_max(sAx); sz = warp_max(sz);
    __syncthreads();
    // ------------------------------------------------ dual residual K x - b + A^T y_o (lanes over nodes)
    double rd = 0.0, sKx = 0.0, sAy = 0.0, sq = 0.0;
    for (int64_t f = lane; f < nf; f += NT) {
      const int64_t i = f + 1;
      const bool right = i < n - 1;
      const ElemK KL = load_elem(d, o + i - 1), KR = load_elem(d, o + (right ? i : i - 1));
      double kx[6] = {0, 0, 0, 0, 0, 0};
      for (int a = 0; a < 6; ++a) {
        if (G.dof(i, a)) continue;
        double s = 0.0;
        for (int b = 0; b < 6; ++b) {
          if (!G.dof(i, b)) s += (k_bb(KL, a, b) + (right ? k_aa(KR, a, b) : 0.0)) * Yr[(6 * f + b) * zp];
          if (f > 0 && !G.dof(i - 1, b)) s += k_ab(KL, b, a) * Yr[(6 * (f - 1) + b) * zp];
          if (right && !G.dof(i + 1, b)) s += k_ab(KR, a, b) * Yr[(6 * (f + 1) + b) * zp];
        }
        kx[a] = s;
      }
      double ay[3] = {0, 0, 0};
      int lo = 0, hi = nc;
      while (lo < hi) { const int mid = (lo + hi) >> 1; if (d.ct_node[cb + mid] < i) lo = mid + 1; else hi = mid; }
      for (int c = lo; c < nc && d.ct_node[cb + c] == i; ++c)
        for (int a = 0; a < 3; ++a) ay[a] += yo[c] * d.ct_n[3 * (cb + c) + a];
      for (int a = 0; a < 6; ++a) {
        if (G.dof(i, a)) continue;
        const double aya = a < 3 ? ay[a] : 0.0;
        const double bq = b0[6 * f + a];
        rd = fmax(rd, fabs(kx[a] - bq + aya));
        sKx = fmax(sKx, fabs(kx[a]));
        sAy = fmax(sAy, fabs(aya));
        sq = fmax(sq, fabs(bq));
      }
    }
    rd = warp_max(rd); sKx = warp_max(sKx); sAy = warp_max(sAy); sq = warp_max(sq);
    const bool stop = rp <= eps + eps * fmax(sAx, sz) && rd <= eps + eps * fmax(sKx, fmax(sAy, sq));
    if (stop) { ++it; break; }
    __syncthreads();
  }
  __syncthreads();
  // ---------------------------------------------------------------- result
  for (int64_t k = lane; k < 6 * nf; k += NT) b0[k] = Yr[k * zp];
  for (int c = lane; c < nc; c += NT) d.ct_y[cb + c] = -yo[c];
  if (lane == 0) {
    d.st_nact[r] = 0;           // the step kernels take x as the whole step
    d.st_mx[r] = 0ull;          // the step's largest node translation is taken afresh
    d.st_qpit[r] += it;
  }
}

// phases of one Newton step: 0 check + right-hand sides, 1 factor, 2 substitute, 3 contact
// forces, 4 step and state update
// The work lists of the pass, after the convergence test: one block scans the robots in solve
// order (still iterating, contact count) and writes every list in that order.
constexpr int WLT = 1024;
__global__ void __launch_bounds__(WLT) build_lists_kernel(Dev d) {
  __shared__ int sTot[WLT / NT][4];
  __shared__ int sBase[4];
  const int t = threadIdx.x, lane = t % NT, wv = t / NT;
  if (t < 4) sBase[t] = 0;
  __syncthreads();
  for (int i0 = 0; i0 < d.B; i0 += WLT) {
    const int i = i0 + t;
    int r = 0, v[4] = {0, 0, 0, 0};   // active, small LCP, wide LCP, substitution passes
    if (i < d.B) {
      r = d.solve_order[i];
      if (!d.st_done[r]) {
        const int nc = d.st_nc[r];
        v[0] = 1;
        v[1] = nc <= LCPM ? 1 : 0;
        v[2] = nc > LCPM ? 1 : 0;
        v[3] = nc > 0 ? (nc + NT) / NT : 0;   // ceil((1 + nc) / NT)
      }
    }
    int ex[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      int x = v[f];
#pragma unroll
      for (int o = 1; o < NT; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
      }
      if (lane == NT - 1) sTot[wv][f] = x;
      ex[f] = x - v[f];
    }
    __syncthreads();
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      int b = sBase[f];
      for (int u = 0; u < wv; ++u) b += sTot[u][f];
      ex[f] += b;
    }
    if (v[0]) d.wl[WL_ACT * d.B + ex[0]] = r;
    if (v[1]) d.wl[WL_SMALL * d.B + ex[1]] = r;
    if (v[2]) d.wl[WL_WIDE * d.B + ex[2]] = r;
    for (int p = 0; p < v[3]; ++p) d.wl_sub[ex[3] + p] = r | (p << 24);
    __syncthreads();
    if (t < 4) {
      int b = 0;
      for (int u = 0; u < WLT / NT; ++u) b += sTot[u][t];
      sBase[t] += b;
    }
    __syncthreads();
  }
  if (t == 0) {
    d.wl_cnt[WL_ACT] = sBase[0];
    d.wl_cnt[WL_SMALL] = sBase[1];
    d.wl_cnt[WL_WIDE] = sBase[2];
    d.wl_cnt[WL_SUB] = sBase[3];
    d.wl_cnt[WL_BIG] = 0;
  }
}

// phase 3 in two parts on disjoint robot lists, which may run on two streams: the LDS LCP,
// and the wide LCP followed by its big-set rerun
void launch_lcp_small(const Dev& d, hipStream_t s) {
  if (!d.qp_admm) hipLaunchKernelGGL(update_kernel, dim3(d.B), dim3(NT), 0, s, d);
}
void launch_lcp_wide(const Dev& d, hipStream_t s) {
  if (d.qp_admm) return;
  if (d.cap > LCPM) hipLaunchKernelGGL(update_wide_kernel, dim3(d.B), dim3(NT), 0, s, d);
  if (d.cap > NPW) hipLaunchKernelGGL(update_big_kernel, dim3(d.B), dim3(NT), 0, s, d);
}

void launch_solve_phase(const Dev& d, int phase, hipStream_t s) {
  switch (phase) {
    case 0:
      hipLaunchKernelGGL(check_rhs_kernel, dim3(d.B), dim3(NT), 0, s, d);
      hipLaunchKernelGGL(build_lists_kernel, dim3(1), dim3(WLT), 0, s, d);
      break;
    case 1:
      if (d.qp_admm) hipLaunchKernelGGL(admm_kernel, dim3(d.B), dim3(NT), 0, s, d);
      else hipLaunchKernelGGL(factor_kernel, dim3(d.B), dim3(4 * NT), 0, s, d);
      break;
    case 2:
      if (!d.qp_admm)
        hipLaunchKernelGGL(subst_kernel, dim3(d.B * ((d.cap + NT) / NT)), dim3(2 * NT), 0, s, d);
      break;
    case 3:
      launch_lcp_small(d, s);
      launch_lcp_wide(d, s);
      break;
    default:
      if (d.qp_admm)
        hipLaunchKernelGGL(step_dx_kernel, dim3((unsigned)((d.Ntot + 255) / 256)), dim3(256), 0, s, d);
      else {
        hipLaunchKernelGGL(add_forces_kernel, dim3((unsigned)((d.Ntot + 255) / 256)), dim3(256), 0, s, d);
        hipLaunchKernelGGL(step_solve_kernel, dim3((unsigned)((d.B + SSR - 1) / SSR)), dim3(64), 0, s, d);
      }
      hipLaunchKernelGGL(step_apply_kernel, dim3((unsigned)((d.Ntot + 255) / 256)), dim3(256), 0, s, d);
      break;
  }
}

void launch_gather(const Dev& d, hipStream_t s) {
  hipLaunchKernelGGL(gather_kernel, dim3(d.B), dim3(NT), 0, s, d);
}

}  // namespace accfem
