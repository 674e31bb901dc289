// HIP kernels and the C ABI of the batched backward-Euler contact step.
//
// One workgroup per world: the world's bodies, rows, Schur matrix and factor
// live in LDS for the whole fused step (contact refresh, Newton loop with
// step length and best-iterate selection, finalisation), so a step is one
// kernel launch for the whole batch.  The adjoint kernel back-solves the
// factor stored by the forward launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <cstring>
#include <string>
#include <vector>

#include "newton.hpp"
#include "ostrich.h"

namespace {

thread_local std::string g_err = "";

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_OK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(OSTRICH_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct GpuTeam {
  static constexpr bool kGlobal = false;  // workspace entirely in LDS
  // whether the rim-circle contact terms are compiled in: only batches with a
  // rim-circle slot run the kernels that carry them (the *Rim team types)
  static constexpr bool kRim = false;
  __device__ int rank() const { return threadIdx.x; }
  __device__ int size() const { return blockDim.x; }
  __device__ void sync() const { __syncthreads(); }
  // The first wavefront alone: its width, a sync among its lanes (LDS
  // operations of a wavefront complete in order; the fences keep the compiler
  // from moving accesses across), and a max over its lanes.
  __device__ int wsize() const { return 64; }
  __device__ void wsync() const {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  __device__ double wmax(double v) const {
    for (int off = 32; off > 0; off >>= 1) {
      double o = __shfl_xor(v, off, 64);
      v = o > v ? o : v;
    }
    return v;
  }
  // v of lane src (uniform) in every lane
  __device__ double bcast(double v, int src) const {
    int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
  }
  // Sum over the team: a butterfly within each 64-lane wavefront, then the
  // wavefront sums in wavefront order; every thread returns the same value.
  __device__ double sum(double v, double* scratch) const {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    int nw = (blockDim.x + 63) >> 6;
    if (nw == 1) return v;
    if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += scratch[i];
    __syncthreads();
    return s;
  }
  // Butterfly sum of the values held by the first wavefront (threads 0..63),
  // broadcast to the team: the result does not depend on the team size.
  __device__ double sum64(double v, double* scratch) const {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (blockDim.x == 64) return v;
    if (threadIdx.x == 0) scratch[0] = v;
    __syncthreads();
    double r = scratch[0];
    __syncthreads();
    return r;
  }
  __device__ int imax(int v, double* scratch) const {
    for (int off = 32; off > 0; off >>= 1) {
      int o = __shfl_xor(v, off, 64);
      v = o > v ? o : v;
    }
    int nw = (blockDim.x + 63) >> 6;
    if (nw == 1) return v;
    if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = (double)v;
    __syncthreads();
    int r = v;
    for (int i = 0; i < nw; ++i) r = (int)scratch[i] > r ? (int)scratch[i] : r;
    __syncthreads();
    return r;
  }
};

// Team whose workspace is (partly) in device memory.  A workgroup barrier
// orders LDS only, so at each sync a wave first waits for its own
// vector-memory operations (its stores are then in L2) and afterwards
// invalidates its CU's vector L1 (agent-scope acquire), so that no lane reads
// a line cached before another lane's store.
struct GpuTeamG : GpuTeam {
  static constexpr bool kGlobal = true;
  __device__ void sync() const {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __device__ void wsync() const {
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __device__ double sum64(double v, double* scratch) const {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (blockDim.x == 64) return v;
    if (threadIdx.x == 0) scratch[0] = v;
    sync();
    double r = scratch[0];
    sync();
    return r;
  }
  __device__ int imax(int v, double* scratch) const {
    for (int off = 32; off > 0; off >>= 1) {
      int o = __shfl_xor(v, off, 64);
      v = o > v ? o : v;
    }
    int nw = (blockDim.x + 63) >> 6;
    if (nw == 1) return v;
    if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = (double)v;
    sync();
    int r = v;
    for (int i = 0; i < nw; ++i) r = (int)scratch[i] > r ? (int)scratch[i] : r;
    sync();
    return r;
  }
};
struct GpuTeamRim : GpuTeam {
  static constexpr bool kRim = true;
};
struct GpuTeamGRim : GpuTeamG {
  static constexpr bool kRim = true;
};

// Launch shape of one bucket of worlds: the worlds of the list are taken by
// workgroups in turn (persistent when the grid is smaller than the list).
struct Launch {
  const int32_t* wlist;  // world ids of the bucket
  int nlist;
  int split;             // ost::SPLIT_LDS or ost::SPLIT_GLOBAL
  double* gscr;          // SPLIT_GLOBAL: per-workgroup slices of gstride doubles
  size_t gstride;
  const int32_t* nlist_dev;  // not null: the list length is read from device memory here
  int32_t* defer;        // not null: a world whose active contacts exceed the carve is appended to
                         // defer[1..] (defer[0] counts them) for a launch with the full carve
  int32_t* hist;         // not null: per world, the active contacts and Newton iterations of its step
};

// Number of worlds of a launch's list.
__device__ __forceinline__ int list_len(const Launch& L) { return L.nlist_dev ? *L.nlist_dev : L.nlist; }

// Hand world w to the launch that follows (one thread of the team).
__device__ __forceinline__ void defer_world(const Launch& L, int w) {
  if (L.defer && threadIdx.x == 0) L.defer[1 + atomicAdd(L.defer, 1)] = w;
}

// kRest marks the launch over the deferred worlds of a tiered bucket (the same
// code under its own name, so that profiles tell the two launches apart).
template <class TeamT, bool kKrylov, bool kRest = false>
__global__ void __launch_bounds__(256, 2) k_forward(ost::Batch B, ost::Params P, ost::Caps caps, Launch L,
                                                 const double* q_prev, const double* u_prev, const double* lam_prev,
                                                 const double* ctrl, double* q_next, double* u_next,
                                                 double* lam_next, int32_t* act_slot, int32_t* n_act,
                                                 int32_t* status, int32_t* iters, double* resnorm, double* tape,
                                                 const int64_t* tape_off) {
  extern __shared__ __align__(16) char smem[];
  TeamT t;
  // the on-chip instantiation carves with a constant split, so that every
  // workspace pointer is known to address LDS
  ost::WorldMem M = TeamT::kGlobal
                        ? ost::carve(smem, caps, blockDim.x, L.split, L.gscr ? L.gscr + blockIdx.x * L.gstride : nullptr)
                        : ost::carve(smem, caps, blockDim.x, ost::SPLIT_LDS, nullptr);
  const int n = list_len(L);
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const int w = L.wlist[i];
    if (!ost::forward_world<TeamT, kKrylov>(t, B, P, caps, w, q_prev, u_prev, lam_prev, ctrl, q_next, u_next, lam_next,
                                            act_slot, n_act, status, iters, resnorm, tape, tape_off, M, L.hist))
      defer_world(L, w);
    __syncthreads();
  }
}

template <class TeamT, bool kRest = false>
__global__ void __launch_bounds__(256, 2) k_adjoint(ost::Batch B, ost::Params P, ost::Caps caps, Launch L,
                                                 const double* q_prev, const double* u_prev, const double* ctrl,
                                                 const double* u_next, const double* lam_next, const double* tape,
                                                 const int64_t* tape_off, const double* gq_next,
                                                 const double* gu_next, double* gq_prev, double* gu_prev,
                                                 double* g_ctrl, int refine, double* g_mass, double* g_mu,
                                                 double* g_kp, int32_t* adj_status) {
  extern __shared__ __align__(16) char smem[];
  TeamT t;
  // the on-chip instantiation carves with a constant split, so that every
  // workspace pointer is known to address LDS
  ost::WorldMem M = TeamT::kGlobal
                        ? ost::carve(smem, caps, blockDim.x, L.split, L.gscr ? L.gscr + blockIdx.x * L.gstride : nullptr,
                                      true)
                        : ost::carve(smem, caps, blockDim.x, ost::SPLIT_LDS, nullptr, true);
  const int n = list_len(L);
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const int w = L.wlist[i];
    if (!ost::adjoint_world(t, B, P, caps, w, q_prev, u_prev, ctrl, u_next, lam_next, tape, tape_off, gq_next,
                            gu_next, gq_prev, gu_prev, g_ctrl, refine, M, g_mass, g_mu, g_kp, adj_status))
      defer_world(L, w);
    __syncthreads();
  }
}

// Launch plan of one bucket: its worlds ordered by an estimated cost, the most
// expensive first (so that the longest worlds do not start last), and split
// into those whose active contacts fit a first carve of nc1 contacts and the
// others (nc1 = 0: one list).  The estimate of a forward step is
// (iterations + 1) m^2 from the world's previous step (hist; zero before its
// first step), with m from nact_now (indexed like worlds) when given, that of
// an adjoint step m^2 from its tape.  The lists are
// permutations of the bucket's worlds (their order within a cost class is that
// of the atomics); per-world results do not depend on them.  plan: [0] count of
// the first list, [1] of the second, [2, 2 + n) the first list, [2 + n,
// 2 + 2 n) the second, and [2 + 2 n, 2 + 3 n) room for nact_now.
__global__ void __launch_bounds__(1024) k_plan(ost::Batch B, const int32_t* worlds, int n, const int32_t* hist,
                                              const int32_t* nact_now, const double* tape, const int64_t* tape_off,
                                              int nc1, int32_t* plan) {
  __shared__ int cnt[2][32];
  __shared__ int pos[2][32];
  for (int i = threadIdx.x; i < 64; i += blockDim.x) cnt[i >> 5][i & 31] = 0;
  __syncthreads();
  auto classify = [&](int i, int& cls, int& bin) {
    const int w = worlds[i];
    const int j0 = B.joint_off[w], j1 = B.joint_off[w + 1];
    int nsv = 0;
    for (int j = j0; j < j1; ++j) nsv += (B.joint_act[j] == 2 || B.joint_act[j] == 3 || B.joint_act[j] == 4);
    const long base = 5L * (j1 - j0) + nsv;
    long m, nact, cost;
    if (tape) {
      const double* tr = tape + tape_off[w + 1] - 4;
      m = tr[2] == 1.0 ? (long)tr[1] : base + 3L * B.contact_cap[w];
      nact = (m - base) / 3;
      cost = m * m;
    } else {
      nact = nact_now ? nact_now[i] : (hist ? hist[2 * w] : 0);
      m = base + 3 * nact;
      cost = (long)((hist ? hist[2 * w + 1] : 0) + 1) * m * m;
    }
    cls = nc1 > 0 && nact > nc1 ? 1 : 0;
    bin = cost > 1 ? 63 - __builtin_clzll((unsigned long long)cost) : 0;
    bin = bin > 31 ? 31 : bin;
  };
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    int c, b;
    classify(i, c, b);
    atomicAdd(&cnt[c][b], 1);
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int c = 0; c < 2; ++c) {
      int run = 0;
      for (int b = 31; b >= 0; --b) {  // costliest class first
        pos[c][b] = run;
        run += cnt[c][b];
      }
      plan[c] = run;
    }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    int c, b;
    classify(i, c, b);
    plan[2 + c * n + atomicAdd(&pos[c][b], 1)] = worlds[i];
  }
}

// Active contacts at q- of each world of a list (the refresh's activation
// test; terrain slots counted active), capped at the world's contact cap:
// out[i] for worlds[i].  One 64-thread workgroup per world.
__global__ void __launch_bounds__(64) k_count_active(ost::Batch B, ost::Params P, const int32_t* worlds,
                                                     const double* q_prev, const double* u_prev,
                                                     const int32_t* hist, int32_t* out) {
  const int w = worlds[blockIdx.x];
  const ost::WorldRef R = ost::world_ref(B, w);
  int nt = 0;
  int c = ost::count_active(B, P, R, q_prev, u_prev, threadIdx.x, 64, &nt);
  for (int off = 32; off > 0; off >>= 1) {
    c += __shfl_xor(c, off, 64);
    nt += __shfl_xor(nt, off, 64);
  }
  // terrain slots: their contacts are only known after the step's mesh search,
  // so the world's contact count of its previous step stands in for them (at
  // most one per terrain slot); a world that then has more than the first
  // carve holds is deferred to the full carve by the step itself
  if (nt > 0) c += hist ? (hist[2 * w] < nt ? hist[2 * w] : nt) : nt;
  if (threadIdx.x == 0) out[blockIdx.x] = c < R.cap ? c : R.cap;
}

// Plain path (the comparison baseline): one launch for a world's set-up, one
// per Newton iteration and one for its finalisation, with the world's
// workspace in device memory between launches.  The arithmetic is that of the
// fused kernel, so the results are the same bits.
__global__ void __launch_bounds__(256) k_plain_begin(ost::Batch B, ost::Params P, ost::Caps caps, int w,
                                                     const double* q_prev, const double* u_prev,
                                                     const double* lam_prev, const double* ctrl, char* ws) {
  GpuTeamGRim t;
  ost::WorldMem M = ost::carve(ws, caps, blockDim.x);
  ost::WorldRef R = ost::world_ref(B, w);
  ost::FwState S;
  ost::fw_begin(t, B, P, R, q_prev, u_prev, lam_prev, ctrl, M, S);
  t.sync();
  if (threadIdx.x == 0) ost::fw_store(M, S);
}

__global__ void __launch_bounds__(256) k_plain_iteration(ost::Batch B, ost::Params P, ost::Caps caps, int w,
                                                         const double* ctrl, char* ws, int k) {
  GpuTeamGRim t;
  ost::WorldMem M = ost::carve(ws, caps, blockDim.x);
  ost::WorldRef R = ost::world_ref_after(B, M, w);
  ost::FwState S = ost::fw_load(M);
  t.sync();
  ost::fw_iteration(t, B, P, R, ctrl, M, S, k);
  t.sync();
  if (threadIdx.x == 0) ost::fw_store(M, S);
}

__global__ void __launch_bounds__(256) k_plain_end(ost::Batch B, ost::Params P, ost::Caps caps, int w,
                                                   const double* ctrl, double* q_next, double* u_next,
                                                   double* lam_next, int32_t* act_slot, int32_t* n_act,
                                                   int32_t* status, int32_t* iters, double* resnorm, double* tape,
                                                   const int64_t* tape_off, char* ws) {
  GpuTeamGRim t;
  ost::WorldMem M = ost::carve(ws, caps, blockDim.x);
  ost::WorldRef R = ost::world_ref_after(B, M, w);
  ost::FwState S = ost::fw_load(M);
  t.sync();
  ost::fw_end(t, B, P, R, w, ctrl, q_next, u_next, lam_next, act_slot, n_act, status, iters, resnorm, tape, tape_off,
              M, S);
}

// Measurement: algorithmic FP64 flops of the forward steps just taken, from
// each world's rows m = 5 joints + servo rows + 3 contacts and its Newton
// iteration count k (Sec. III-C: one Schur-complement factor and solve per
// iteration).  acc[0] takes the dense per-iteration count k (m^3/3 + 14 m^2 +
// 170 m) of the roofline; acc[2] the finer count of this implementation's
// operations: k (26 m^2 + 2 m^3 / 3 + 800 m) + 400 m for the set-up, plus the
// factor at the returned iterate when a tape is written (24 m^2 + 2 m^3 / 3).
// One workgroup sums in a fixed order.
__global__ void k_flops(ost::Batch B, const int32_t* n_act, const int32_t* iters, int with_tape, double* acc) {
  __shared__ double part[2][256];
  double s = 0.0, f = 0.0;
  for (int w = threadIdx.x; w < B.n_worlds; w += blockDim.x) {
    int nsv = 0;
    for (int j = B.joint_off[w]; j < B.joint_off[w + 1]; ++j) nsv += (B.joint_act[j] == 2 || B.joint_act[j] == 3 || B.joint_act[j] == 4);
    const double m = 5.0 * (B.joint_off[w + 1] - B.joint_off[w]) + nsv + 3.0 * n_act[w];
    s += iters[w] * (m * m * m / 3.0 + 14.0 * m * m + 170.0 * m);
    const double per_it = 24.0 * m * m + 2.0 * m * m * m / 3.0 + 2.0 * m * m + 800.0 * m;
    f += iters[w] * per_it + 400.0 * m + (with_tape ? 24.0 * m * m + 2.0 * m * m * m / 3.0 : 0.0);
  }
  part[0][threadIdx.x] = s;
  part[1][threadIdx.x] = f;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0, u = 0.0;
    for (int i = 0; i < (int)blockDim.x; ++i) {
      t += part[0][i];
      u += part[1][i];
    }
    acc[0] += t;
    acc[2] += u;
  }
}

// Algorithmic bytes of one adjoint step of every world (Sec. III-D: one solve
// with the stored factor).  acc[1] takes the roofline's count: the states read
// and written (2 x 13 doubles per body), the multipliers read, and a
// triangular factor of the world's m rows, m (m + 1) / 2 doubles.  acc[3] the
// bytes of this implementation: the factor's band as the tape stores it
// (rows m and half band bw from the tape's trailer), the states and
// multipliers read, the cotangents read and written, and the control
// cotangents written.
__global__ void k_abytes(ost::Batch B, const double* tape, const int64_t* tape_off, double* acc) {
  __shared__ double part[2][256];
  double s = 0.0, f = 0.0;
  for (int w = threadIdx.x; w < B.n_worlds; w += blockDim.x) {
    const double* tr = tape + tape_off[w + 1] - 4;
    const double m = tr[1], bw = tr[3] < tr[1] - 1 ? tr[3] : tr[1] - 1;
    const double band = m > 0 ? m * (2.0 * bw + 1.0) - bw * (bw + 1.0) : 0.0;
    const double nb = B.body_off[w + 1] - B.body_off[w];
    const double nl = B.lam_off[w + 1] - B.lam_off[w], nc = B.ctrl_off[w + 1] - B.ctrl_off[w];
    s += 8.0 * (2.0 * 13.0 * nb + nl + m * (m + 1.0) / 2.0);
    f += 8.0 * (band + 4 + 13.0 * nb + 6.0 * nb + nl + 2.0 * 13.0 * nb + nc);
  }
  part[0][threadIdx.x] = s;
  part[1][threadIdx.x] = f;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0, u = 0.0;
    for (int i = 0; i < (int)blockDim.x; ++i) {
      t += part[0][i];
      u += part[1][i];
    }
    acc[1] += t;
    acc[3] += u;
  }
}

// controls of every step: ctrl[k, c] = sum_j basis[k, j] knots[c, j]
__global__ void k_ctrl(const double* basis, const double* knots, int T, int K, int nctrl, double* ctrl) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T * nctrl) return;
  int k = i / nctrl, c = i - k * nctrl;
  double s = 0.0;
  for (int j = 0; j < K; ++j) s += basis[k * K + j] * knots[c * K + j];
  ctrl[i] = s;
}

__global__ void k_fill(double* p, long n, double v) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Body row of world w's loss body, or -1 (status bit ST_LOSS_BODY) when
// loss_body[w] is not one of the world's bodies.
__device__ int loss_row(const int32_t* body_off, const int32_t* loss_body, int w, int32_t* status) {
  const int lb = loss_body[w];
  if (lb >= 0 && lb < body_off[w + 1] - body_off[w]) return body_off[w] + lb;
  if (status) status[w] |= ost::ST_LOSS_BODY;
  return -1;
}

// loss |xy(loss_body) - target|^2 and its cotangent on q_T (NaN loss and no
// cotangent for a loss body outside its world)
__global__ void k_loss(const int32_t* body_off, int W, const double* qT, const int32_t* loss_body,
                       const double* target, const double* loss_grad, double* loss, double* gq, int32_t* status) {
  int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  const int b = loss_row(body_off, loss_body, w, status);
  if (b < 0) {
    if (loss) loss[w] = NAN;
    return;
  }
  double dx = qT[7 * b] - target[2 * w], dy = qT[7 * b + 1] - target[2 * w + 1];
  if (loss) loss[w] = dx * dx + dy * dy;
  if (gq) {
    double g = loss_grad ? loss_grad[w] : 1.0;
    gq[7 * b] = 2.0 * dx * g;
    gq[7 * b + 1] = 2.0 * dy * g;
  }
}

// Shaped loss of the optimisation workload (device copy of ostrich_loss).
struct LossDev {
  double w_pos, w_head, w_vel, w_ctrl, w_track, w_yaw;
  const double* goal;
  const double* ref;
};

// wt (1 - cos(psi - rho)) of a body's yaw psi (the heading of its x axis in the
// ground plane) from its unit quaternion (x, y, z, w), with the cotangent on
// the quaternion added to dq[3..6]: with R00 = 1 - 2 (y^2 + z^2), R10 =
// 2 (x y + w z) and n = |(R00, R10)|, cos(psi - rho) = (R00 cos rho + R10 sin rho) / n.
__device__ double yaw_term(const double* qb, double rho, double wt, double* dq) {
  const double x = qb[3], y = qb[4], z = qb[5], w = qb[6];
  const double r00 = 1.0 - 2.0 * (y * y + z * z), r10 = 2.0 * (x * y + w * z);
  const double n2 = r00 * r00 + r10 * r10, n = ::sqrt(n2);
  const double ca = ::cos(rho), sa = ::sin(rho);
  const double c = (r00 * ca + r10 * sa) / n;
  const double sg = (ca * r10 - sa * r00) / (n2 * n);
  const double f00 = -wt * r10 * sg, f10 = wt * r00 * sg;  // d/dR00, d/dR10 of wt (1 - c)
  dq[3] += f10 * 2.0 * y;
  dq[4] += f00 * (-4.0 * y) + f10 * 2.0 * x;
  dq[5] += f00 * (-4.0 * z) + f10 * 2.0 * w;
  dq[6] += f10 * 2.0 * z;
  return wt * (1.0 - c);
}

// Terms of state k (1 <= k <= T) of each world's shaped loss: tracking and yaw
// alignment against the reference of step k and, at k = T, the final position,
// heading and velocity.  Adds them to loss[w] (if loss) and their cotangents,
// times loss_grad[w], to the state's gq, gu (if gq).
__global__ void k_state_loss(const int32_t* body_off, int W, const double* q, const double* u,
                             const int32_t* loss_body, LossDev L, int k, int T, const double* loss_grad,
                             double* loss, double* gq, double* gu, int32_t* status) {
  int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  const int b = loss_row(body_off, loss_body, w, status);
  if (b < 0) {
    if (loss) loss[w] = NAN;
    return;
  }
  const double* qb = q + 7 * b;
  const double* ub = u + 6 * b;
  double dq[7] = {0, 0, 0, 0, 0, 0, 0}, du[3] = {0, 0, 0};
  double s = 0.0;
  const double iT = 1.0 / T;
  if (L.w_track != 0.0 || L.w_yaw != 0.0) {
    const double* r = L.ref + 3 * ((size_t)(k - 1) * W + w);
    const double ex = qb[0] - r[0], ey = qb[1] - r[1];
    const double wt = L.w_track * iT;
    s += wt * (ex * ex + ey * ey);
    dq[0] += 2.0 * wt * ex;
    dq[1] += 2.0 * wt * ey;
    if (L.w_yaw != 0.0) s += yaw_term(qb, r[2], L.w_yaw * iT, dq);
  }
  if (k == T) {
    const double* gl = L.goal + 3 * w;
    const double ex = qb[0] - gl[0], ey = qb[1] - gl[1];
    s += L.w_pos * (ex * ex + ey * ey);
    dq[0] += 2.0 * L.w_pos * ex;
    dq[1] += 2.0 * L.w_pos * ey;
    if (L.w_head != 0.0) s += yaw_term(qb, gl[2], L.w_head, dq);
    s += L.w_vel * (ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2]);
    for (int i = 0; i < 3; ++i) du[i] = 2.0 * L.w_vel * ub[i];
  }
  if (loss) loss[w] += s;
  if (gq) {
    const double g = loss_grad ? loss_grad[w] : 1.0;
    for (int i = 0; i < 7; ++i) gq[7 * b + i] += g * dq[i];
    for (int i = 0; i < 3; ++i) gu[6 * b + i] += g * du[i];
  }
}

// Control regulariser of the shaped loss, wt sum_{k<T} |a_k|^2 over each
// world's controls, added to loss[w].
__global__ void k_ctrl_loss(const int32_t* ctrl_off, int W, const double* ctrl, int T, int nctrl, double wt,
                            double* loss) {
  int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  double s = 0.0;
  for (int k = 0; k < T; ++k)
    for (int c = ctrl_off[w]; c < ctrl_off[w + 1]; ++c) {
      const double a = ctrl[(size_t)k * nctrl + c];
      s += a * a;
    }
  loss[w] += wt * s;
}

// Its cotangent on the controls of one step: g_ctrl[c] += 2 wt a[c] loss_grad[w].
__global__ void k_ctrl_reg_grad(const int32_t* ctrl_off, int W, const double* ctrl_k, double wt,
                                const double* loss_grad, double* gctrl) {
  int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  const double g = loss_grad ? loss_grad[w] : 1.0;
  for (int c = ctrl_off[w]; c < ctrl_off[w + 1]; ++c) gctrl[c] += 2.0 * wt * ctrl_k[c] * g;
}

__global__ void k_gknots(const double* basis, const double* gctrl, int k, int K, int nctrl, double* g_knots) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nctrl * K) return;
  int c = i / K, j = i - c * K;
  g_knots[i] += basis[k * K + j] * gctrl[c];
}

__global__ void k_or(int32_t* acc, const int32_t* st, int W) {
  int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w < W) acc[w] |= st[w];
}

__global__ void k_zero_i(int32_t* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

inline int nblk(long n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

namespace {
// One bucket of worlds with similar row capacity, and its launch choice.
struct Bucket {
  ost::Caps caps{0, 0, 0, 0, 0, 0};
  std::vector<int32_t> worlds;  // host copy of the world ids
  int32_t* d_worlds = nullptr;
  int team = 128;
  int split = ost::SPLIT_LDS;
  size_t lds = 0;                // forward kernel's LDS per workgroup
  size_t lds_adj = 0;            // adjoint kernel's (adds the Krylov workspace)
  int slots = 0;                // SPLIT_GLOBAL: workgroups of the persistent grid
  double* gscr = nullptr;
  size_t gstride = 0;
  bool tuned = false;
  // Tiered on-chip launch: a first launch carves for at most caps1.nc active
  // contacts (more workgroups per CU), and the worlds with more are done by a
  // second, persistent launch with the full carve.
  bool tier = false;
  ost::Caps caps1{0, 0, 0, 0, 0, 0};
  size_t lds1 = 0, lds1_adj = 0;
  int grid2 = 0;
  int32_t* d_defer = nullptr;  // [0] deferred count, [1..] their world ids
  int32_t* d_plan = nullptr;   // launch plan (k_plan): two counts and two world lists
  hipStream_t side = nullptr;  // tiered: the full-carve launch runs here beside the first one
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

// Row capacity edges of the buckets: a world with row cap mr goes to the first
// bucket whose edge is >= mr.
const int kEdges[] = {16, 32, 64, 96, 128, 192, 256, 384, 1 << 30};
const int kPlainTeam = 128;
}  // namespace

struct ostrich_ctx {
  ost::Batch B;
  ost::Params P;
  ost::Caps caps;  // maxima over the batch
  int team;
  int schedule;
  int tier_contacts;  // ostrich_params::tier_contacts
  bool rim = false;   // the batch has rim-circle slots: launch the kernels with those terms
  size_t lds_limit;
  int n_cu;
  int W, NB, NL, NS, NCTRL;
  int refine;
  std::vector<int32_t> body_off_h;
  std::vector<ost::Caps> wcaps;  // per world
  std::vector<Bucket> buckets;
  Bucket all;  // every world, shaped for the largest: launches over caller-given world lists
  char* plain_ws = nullptr;  // one world's workspace for the plain path
  // concurrent buckets: one stream per bucket, forked from and joined to the caller's stream
  std::vector<hipStream_t> bstreams;
  hipEvent_t ev_fork = nullptr;
  std::vector<hipEvent_t> ev_join;
  // measurement of the forward and adjoint launches (ostrich_ctx_timing)
  bool timing = false;
  std::vector<hipEvent_t> ev;  // forward start / stop pairs
  size_t n_ev = 0;
  double* d_flops = nullptr;  // forward flops, adjoint bytes (roofline counts), then the same by finer counts
  std::vector<hipEvent_t> eva;  // adjoint start / stop pairs
  size_t n_eva = 0;
  int64_t* d_tape_off = nullptr;
  size_t tape_total = 0;  // doubles
  std::map<void*, size_t> allocs;  // device memory held by the context, by allocation
  int32_t* d_hist = nullptr;  // per world: active contacts and Newton iterations of its last forward step
  ~ostrich_ctx() {
    auto free_bucket = [](Bucket& b) {
      if (b.d_worlds) (void)hipFree(b.d_worlds);
      if (b.gscr) (void)hipFree(b.gscr);
      if (b.d_defer) (void)hipFree(b.d_defer);
      if (b.d_plan) (void)hipFree(b.d_plan);
      if (b.side) (void)hipStreamDestroy(b.side);
      if (b.ev_fork) (void)hipEventDestroy(b.ev_fork);
      if (b.ev_join) (void)hipEventDestroy(b.ev_join);
    };
    for (auto& b : buckets) free_bucket(b);
    free_bucket(all);
    if (d_hist) (void)hipFree(d_hist);
    if (plain_ws) (void)hipFree(plain_ws);
    if (d_flops) (void)hipFree(d_flops);
    for (hipStream_t x : bstreams) (void)hipStreamDestroy(x);
    for (hipEvent_t e : ev_join) (void)hipEventDestroy(e);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : eva) (void)hipEventDestroy(e);
    if (d_tape_off) (void)hipFree(d_tape_off);
  }
};

extern "C" const char* ostrich_last_error(void) { return g_err.c_str(); }

static bool is_ptr_ok(const void* p) { return p != nullptr; }

static ost::Caps caps_max(const ost::Caps& a, const ost::Caps& b) {
  return ost::Caps{std::max(a.nb, b.nb), std::max(a.nj, b.nj), std::max(a.ns, b.ns),
                   std::max(a.nc, b.nc), std::max(a.mr, b.mr), std::max(a.nsv, b.nsv)};
}

static bool team_ok(int t) { return t == 64 || t == 128 || t == 256; }

// Device allocations owned by the context, counted for ostrich_ctx_device_bytes.
template <class T> static hipError_t ctx_malloc(ostrich_ctx* ctx, T** p, size_t bytes) {
  hipError_t e = hipMalloc((void**)p, bytes);
  if (e == hipSuccess) ctx->allocs[(void*)*p] = bytes;
  return e;
}
static hipError_t ctx_free(ostrich_ctx* ctx, void* p) {
  if (!p) return hipSuccess;
  ctx->allocs.erase(p);
  return hipFree(p);
}

// Fewest active contacts a tiered first launch carves for.
const int kTierMinContacts = 4;

// Carve of a tiered first launch: the largest contact capacity below the
// bucket's whose adjoint workspace lets more workgroups share a CU than the
// full carve does, up to the limit the kernels' registers set (two wavefronts
// per SIMD).  False when no such carve exists.
static bool tier_caps(const ostrich_ctx* ctx, const Bucket& bk, int team, ost::Caps* out) {
  if (ctx->tier_contacts < 0) return false;
  if (ctx->tier_contacts > 0) {  // a requested count
    if (ctx->tier_contacts >= bk.caps.nc) return false;
    ost::Caps c = bk.caps;
    c.nc = ctx->tier_contacts;
    c.mr = std::min(bk.caps.mr, 5 * bk.caps.nj + bk.caps.nsv + 3 * c.nc);
    *out = c;
    return true;
  }
  const int occ_full = (int)(ctx->lds_limit / std::max<size_t>(1, ost::world_lds_bytes(bk.caps, team, ost::SPLIT_LDS, true)));
  const int occ_max = std::max(1, 8 / (team / 64));
  for (int occ = occ_max; occ > occ_full; --occ)
    for (int nc = bk.caps.nc - 1; nc >= kTierMinContacts; --nc) {
      ost::Caps c = bk.caps;
      c.nc = nc;
      c.mr = std::min(bk.caps.mr, 5 * bk.caps.nj + bk.caps.nsv + 3 * nc);
      if (ost::world_lds_bytes(c, team, ost::SPLIT_LDS, true) * occ <= ctx->lds_limit) {
        *out = c;
        return true;
      }
    }
  return false;
}

// Decide the storage split (and, on chip, the tiering) of a bucket for a team
// size and (re)allocate its device scratch; fails if the world does not fit
// either way.
static int configure_bucket(ostrich_ctx* ctx, Bucket& bk, int team, int split, bool tier = true) {
  size_t lds = ost::world_lds_bytes(bk.caps, team, split);
  size_t lds_adj = ost::world_lds_bytes(bk.caps, team, split, true);
  if (lds_adj > ctx->lds_limit) return fail(OSTRICH_E_UNSUPPORTED, "bucket does not fit in LDS");
  bk.team = team;
  bk.split = split;
  bk.lds = lds;
  bk.lds_adj = lds_adj;
  bk.tier = split == ost::SPLIT_LDS && tier && tier_caps(ctx, bk, team, &bk.caps1);
  if (bk.tier) {
    bk.lds1 = ost::world_lds_bytes(bk.caps1, team, ost::SPLIT_LDS);
    bk.lds1_adj = ost::world_lds_bytes(bk.caps1, team, ost::SPLIT_LDS, true);
    const size_t per_cu = std::max<size_t>(1, ctx->lds_limit / lds_adj);
    bk.grid2 = (int)std::min<size_t>(bk.worlds.size(), per_cu * ctx->n_cu);
    if (!bk.d_defer) HIP_OK(ctx_malloc(ctx, &bk.d_defer, (bk.worlds.size() + 1) * sizeof(int32_t)));
    if (!bk.side) {  // default priority, events without timing
      HIP_OK(hipStreamCreateWithFlags(&bk.side, hipStreamNonBlocking));
      HIP_OK(hipEventCreateWithFlags(&bk.ev_fork, hipEventDisableTiming));
      HIP_OK(hipEventCreateWithFlags(&bk.ev_join, hipEventDisableTiming));
    }
  }
  if (!bk.d_plan) HIP_OK(ctx_malloc(ctx, &bk.d_plan, (3 * bk.worlds.size() + 2) * sizeof(int32_t)));
  if (split == ost::SPLIT_GLOBAL) {
    size_t per_cu = std::max<size_t>(1, ctx->lds_limit / std::max<size_t>(lds, 1));
    per_cu = std::min<size_t>(per_cu, 2048 / team);
    int slots = (int)std::min<size_t>(bk.worlds.size(), per_cu * ctx->n_cu);
    size_t stride = (ost::world_glob_doubles(bk.caps, split) + 31) & ~size_t(31);
    if (!bk.gscr || slots * stride > (size_t)bk.slots * bk.gstride) {
      if (bk.gscr) HIP_OK(ctx_free(ctx, bk.gscr));
      bk.gscr = nullptr;
      HIP_OK(ctx_malloc(ctx, &bk.gscr, sizeof(double) * stride * slots));
    }
    bk.slots = slots;
    bk.gstride = stride;
  }
  return 0;
}

// Default launch choice: the requested team, on chip when it fits.  Without a
// request: 128 threads (two wavefronts), or 256 when a world's on-chip
// workspace leaves room for only one workgroup per CU, so that the one
// workgroup's wavefronts still cover the CU's four SIMDs (terrain robots with
// cylinder wheels: 1.7 x the served world-steps of 128 threads, same bits).
static int default_config(ostrich_ctx* ctx, Bucket& bk) {
  int team = ctx->team;
  if (team == 0) {
    team = 128;
    const size_t l128 = ost::world_lds_bytes(bk.caps, 128, ost::SPLIT_LDS, true);
    if (l128 <= ctx->lds_limit && 2 * l128 > ctx->lds_limit &&
        ost::world_lds_bytes(bk.caps, 256, ost::SPLIT_LDS, true) <= ctx->lds_limit)
      team = 256;
  }
  if (ost::world_lds_bytes(bk.caps, team, ost::SPLIT_LDS, true) <= ctx->lds_limit)
    return configure_bucket(ctx, bk, team, ost::SPLIT_LDS);
  return configure_bucket(ctx, bk, team, ost::SPLIT_GLOBAL);
}

// Device scratch a bucket's launches use: the deferral queue of a tiered
// bucket, and the per-workgroup slices of a bucket kept in device memory
// (slots workgroups of gstride doubles).  The context's own, or slices of the
// static array of the allocation-free entry point.
struct Scratch {
  int32_t* defer;
  double* gscr;
  int slots;
  int32_t* plan;
};
static Scratch own_scratch(const Bucket& bk) { return Scratch{bk.d_defer, bk.gscr, bk.slots, bk.d_plan}; }

// The launch over a tiered bucket's deferred worlds (the full carve).
static Launch launch_deferred(const Scratch& sc) {
  return Launch{sc.defer + 1, 0, ost::SPLIT_LDS, nullptr, 0, sc.defer, nullptr, nullptr};
}

static int grid_of(const Bucket& bk, const Scratch& sc) {
  int n = (int)bk.worlds.size();
  return bk.split == ost::SPLIT_GLOBAL ? std::max(1, std::min(n, sc.slots)) : n;
}
static int grid_of(const Bucket& bk) { return grid_of(bk, own_scratch(bk)); }

// ---------------------------------------------------------------------------
// Scratch of the allocation-free entry point: a file-scope device array (one
// copy per GPU, held until the process ends).  Host code never uses the
// array's name as an address: each device's address comes from
// hipGetSymbolAddress, taken once per device (at context creation, or at the
// entry point's first call on a device) and kept in scratch_dev.
namespace {
constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) char scratch[kScratchBytes];
std::mutex g_scratch_mu;
char* g_scratch_dev[kMaxDevices] = {};

// The current device's copy of the scratch array (set up on first use).
int scratch_dev(char** out) {
  int dev = -1;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(OSTRICH_E_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    HIP_OK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(OSTRICH_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_dev[dev] = (char*)ptr;
  }
  *out = g_scratch_dev[dev];
  return 0;
}

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }
}  // namespace

extern "C" int ostrich_ctx_create(const ostrich_batch* b, const ostrich_params* p, ostrich_ctx** out) {
  if (!b || !p || !out) return fail(OSTRICH_E_ARG, "null argument");
  if (b->n_worlds < 1) return fail(OSTRICH_E_ARG, "n_worlds must be >= 1");
  if (!(p->h > 0.0) || p->k_max < 0 || p->k_min < 0 || p->ls_max < 0 || !(p->tol >= 0.0) || !(p->eps > 0.0) ||
      !(p->delta_reg > 0.0) || !(p->delta_reg_adj > 0.0))
    return fail(OSTRICH_E_ARG, "invalid solver parameters");
  if (p->schedule != OSTRICH_SCHED_FIXED && p->schedule != OSTRICH_SCHED_BUCKETED)
    return fail(OSTRICH_E_ARG, "schedule must be OSTRICH_SCHED_FIXED or OSTRICH_SCHED_BUCKETED");
  const void* need[] = {b->body_off, b->body_mass, b->body_inertia, b->joint_off, b->ctrl_off, b->slot_off,
                        b->obs_off, b->lam_off, b->contact_cap};
  for (const void* q : need)
    if (!is_ptr_ok(q)) return fail(OSTRICH_E_ARG, "null array in batch");
  int team = p->team > 0 ? p->team : 0;  // 0: chosen per bucket (default_config)
  if (team != 0 && !team_ok(team)) return fail(OSTRICH_E_ARG, "team must be 64, 128 or 256");
  const int W = b->n_worlds;
  std::vector<int32_t> bo(W + 1), jo(W + 1), so(W + 1), co(W + 1), lo(W + 1), cap(W);
  HIP_OK(hipMemcpy(bo.data(), b->body_off, (W + 1) * 4, hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(jo.data(), b->joint_off, (W + 1) * 4, hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(so.data(), b->slot_off, (W + 1) * 4, hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(co.data(), b->ctrl_off, (W + 1) * 4, hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(lo.data(), b->lam_off, (W + 1) * 4, hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(cap.data(), b->contact_cap, W * 4, hipMemcpyDeviceToHost));
  std::vector<int32_t> act(std::max(jo[W], 1), 0);
  if (jo[W] > 0) HIP_OK(hipMemcpy(act.data(), b->joint_act, jo[W] * 4, hipMemcpyDeviceToHost));
  bool rim = false;
  if (so[W] > 0) {  // rim circles: a unit axis, and static features only
    if (!is_ptr_ok(b->slot_int) || !is_ptr_ok(b->slot_real)) return fail(OSTRICH_E_ARG, "null slot arrays");
    std::vector<int32_t> si(4 * (size_t)so[W]);
    std::vector<double> sr(9 * (size_t)so[W]);
    HIP_OK(hipMemcpy(si.data(), b->slot_int, si.size() * 4, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(sr.data(), b->slot_real, sr.size() * 8, hipMemcpyDeviceToHost));
    for (int32_t s = 0; s < so[W]; ++s) {
      const double* a = sr.data() + 9 * (size_t)s;
      const double n2 = a[6] * a[6] + a[7] * a[7] + a[8] * a[8];
      if (n2 == 0.0) continue;
      rim = true;
      if (!(std::fabs(n2 - 1.0) <= 1e-12)) return fail(OSTRICH_E_ARG, "slot " + std::to_string(s) +
                                                                         ": a rim circle's axis must be a unit vector");
      if (si[4 * (size_t)s] == 2 || !(a[3] > 0.0))
        return fail(OSTRICH_E_ARG, "slot " + std::to_string(s) +
                                       ": a rim circle needs a positive radius and a static feature");
    }
  }
  std::unique_ptr<ostrich_ctx> ctx(new ostrich_ctx());
  ctx->rim = rim;
  ctx->wcaps.resize(W);
  ost::Caps c{0, 0, 0, 0, 0, 0};
  std::vector<int64_t> toff(W + 1, 0);
  for (int w = 0; w < W; ++w) {
    int nb = bo[w + 1] - bo[w], nj = jo[w + 1] - jo[w], ns = so[w + 1] - so[w];
    if (nb < 1 || nj < 0 || ns < 0 || cap[w] < 0 || co[w + 1] < co[w] || lo[w + 1] < lo[w])
      return fail(OSTRICH_E_ARG, "malformed offsets");
    int nsv = 0;
    for (int j = jo[w]; j < jo[w + 1]; ++j) nsv += (act[j] == 2 || act[j] == 3 || act[j] == 4);
    int nc = std::min(cap[w], ns);
    ost::Caps wc{nb, nj, std::max(ns, 1), std::max(nc, 1), std::max(5 * nj + nsv + 3 * nc, 1), nsv};
    if (wc.mr > ost::kMaxRows)
      return fail(OSTRICH_E_UNSUPPORTED, "world " + std::to_string(w) + " has " + std::to_string(wc.mr) +
                                             " constraint rows, more than " + std::to_string(ost::kMaxRows));
    ctx->wcaps[w] = wc;
    c = caps_max(c, wc);
    toff[w + 1] = toff[w] + (int64_t)ost::tape_doubles_world(wc.mr);
  }
  hipDeviceProp_t prop;
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  HIP_OK(hipGetDeviceProperties(&prop, dev));
  ctx->lds_limit = prop.sharedMemPerBlock;
  ctx->n_cu = std::max(1, prop.multiProcessorCount);
  {  // this device's address of the allocation-free entry point's scratch array
    char* scr = nullptr;
    if (int rc = scratch_dev(&scr)) return rc;
  }
  for (auto f : {(const void*)k_forward<GpuTeam, false>, (const void*)k_adjoint<GpuTeam>,
                 (const void*)k_forward<GpuTeamG, false>, (const void*)k_adjoint<GpuTeamG>,
                 (const void*)k_forward<GpuTeam, false, true>, (const void*)k_adjoint<GpuTeam, true>,
                 (const void*)k_forward<GpuTeamRim, false>, (const void*)k_adjoint<GpuTeamRim>,
                 (const void*)k_forward<GpuTeamGRim, false>, (const void*)k_adjoint<GpuTeamGRim>,
                 (const void*)k_forward<GpuTeamRim, false, true>, (const void*)k_adjoint<GpuTeamRim, true>})
    HIP_OK(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)ctx->lds_limit));
  std::memcpy(&ctx->B, b, sizeof(ost::Batch));
  static_assert(sizeof(ost::Batch) == sizeof(ostrich_batch), "batch layouts differ");
  ctx->P.h = p->h;
  for (int k = 0; k < 3; ++k) ctx->P.g[k] = p->gravity[k];
  ctx->P.tol = p->tol;
  ctx->P.eps = p->eps;
  ctx->P.dg = p->delta_g;
  ctx->P.dreg = p->delta_reg;
  ctx->P.dreg_adj = p->delta_reg_adj;
  ctx->P.d0 = p->delta0;
  ctx->P.kmax = p->k_max;
  ctx->P.kmin = std::min(p->k_min, p->k_max);
  ctx->P.ls_max = p->ls_max;
  ctx->P.refine = p->refine;
  ctx->P.truncate = p->truncate ? 1 : 0;
  if (p->linear_solver != OSTRICH_LIN_LU && p->linear_solver != OSTRICH_LIN_KRYLOV)
    return fail(OSTRICH_E_ARG, "linear_solver must be OSTRICH_LIN_LU or OSTRICH_LIN_KRYLOV");
  if (p->linear_solver == OSTRICH_LIN_KRYLOV)  // switched off: its kernel faulted on the GPU, cause not found
    return fail(OSTRICH_E_UNSUPPORTED, "the matrix-free Krylov Newton step is switched off in this version of the library");
  if (p->krylov_iters < 0) return fail(OSTRICH_E_ARG, "krylov_iters must be >= 0");
  ctx->P.lin = p->linear_solver;
  ctx->P.lin_iters = p->krylov_iters > 0 ? p->krylov_iters : 16;
  ctx->refine = p->refine;
  ctx->tier_contacts = p->tier_contacts;
  ctx->caps = c;
  ctx->team = team;
  ctx->schedule = p->schedule;
  ctx->W = W;
  ctx->NB = bo[W];
  ctx->NL = lo[W];
  ctx->NS = so[W];
  ctx->NCTRL = co[W];
  ctx->body_off_h = bo;
  ctx->tape_total = (size_t)toff[W];
  // buckets: one for the fixed schedule, else by row capacity
  if (p->schedule == OSTRICH_SCHED_FIXED) {
    ctx->buckets.resize(1);
    for (int w = 0; w < W; ++w) ctx->buckets[0].worlds.push_back(w);
    ctx->buckets[0].caps = c;
  } else {
    const int ne = sizeof(kEdges) / sizeof(kEdges[0]);
    std::vector<Bucket> bk(ne);
    for (int w = 0; w < W; ++w) {
      int e = 0;
      while (kEdges[e] < ctx->wcaps[w].mr) ++e;
      bk[e].worlds.push_back(w);
      bk[e].caps = caps_max(bk[e].caps, ctx->wcaps[w]);
    }
    for (auto& x : bk)
      if (!x.worlds.empty()) ctx->buckets.push_back(std::move(x));
  }
  for (auto& x : ctx->buckets) {
    HIP_OK(ctx_malloc(ctx.get(), &x.d_worlds, x.worlds.size() * sizeof(int32_t)));
    HIP_OK(hipMemcpy(x.d_worlds, x.worlds.data(), x.worlds.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    int rc = default_config(ctx.get(), x);
    if (rc) return fail(OSTRICH_E_UNSUPPORTED, "a world with " + std::to_string(x.caps.mr) +
                                                   " rows needs more LDS than a workgroup has");
  }
  for (int w = 0; w < W; ++w) ctx->all.worlds.push_back(w);
  ctx->all.caps = c;
  HIP_OK(ctx_malloc(ctx.get(), &ctx->all.d_worlds, W * sizeof(int32_t)));
  HIP_OK(hipMemcpy(ctx->all.d_worlds, ctx->all.worlds.data(), W * sizeof(int32_t), hipMemcpyHostToDevice));
  if (default_config(ctx.get(), ctx->all))
    return fail(OSTRICH_E_UNSUPPORTED, "the batch does not fit a workgroup");
  HIP_OK(ctx_malloc(ctx.get(), &ctx->plain_ws, ost::world_lds_bytes(c, kPlainTeam) + 256));
  if (ctx->buckets.size() > 1) {  // streams of default priority, events without timing
    HIP_OK(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
    for (size_t i = 0; i < ctx->buckets.size(); ++i) {
      hipStream_t x;
      hipEvent_t e;
      HIP_OK(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
      ctx->bstreams.push_back(x);
      HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      ctx->ev_join.push_back(e);
    }
  }
  HIP_OK(ctx_malloc(ctx.get(), &ctx->d_tape_off, (W + 1) * sizeof(int64_t)));
  HIP_OK(hipMemcpy(ctx->d_tape_off, toff.data(), (W + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
  HIP_OK(ctx_malloc(ctx.get(), &ctx->d_hist, 2 * (size_t)W * sizeof(int32_t)));
  HIP_OK(hipMemset(ctx->d_hist, 0, 2 * (size_t)W * sizeof(int32_t)));
  *out = ctx.release();
  return 0;
}

extern "C" int ostrich_ctx_destroy(ostrich_ctx* ctx) {
  delete ctx;
  return 0;
}

extern "C" size_t ostrich_ctx_device_bytes(const ostrich_ctx* ctx) {
  if (!ctx) return 0;
  size_t n = 0;
  for (const auto& a : ctx->allocs) n += a.second;
  return n;
}

extern "C" int ostrich_ctx_caps(const ostrich_ctx* ctx, int64_t* out) {
  if (!ctx || !out) return fail(OSTRICH_E_ARG, "null argument");
  size_t lds = 0;
  for (const auto& b : ctx->buckets) lds = std::max(lds, b.lds);
  out[0] = ctx->caps.nb;
  out[1] = ctx->caps.nj;
  out[2] = ctx->caps.ns;
  out[3] = ctx->caps.nc;
  out[4] = ctx->caps.mr;
  out[5] = (int64_t)lds;
  return 0;
}

extern "C" int ostrich_ctx_schedule(const ostrich_ctx* ctx, int32_t* out, int32_t max_buckets) {
  if (!ctx) return fail(OSTRICH_E_ARG, "null argument");
  int n = (int)ctx->buckets.size();
  if (out)
    for (int i = 0; i < std::min(n, (int)max_buckets); ++i) {
      const Bucket& b = ctx->buckets[i];
      int32_t* o = out + 8 * i;
      o[0] = b.caps.mr;
      o[1] = (int32_t)b.worlds.size();
      o[2] = b.team;
      o[3] = b.split;
      o[4] = (int32_t)b.lds;
      o[5] = b.tuned ? 1 : 0;
      o[6] = b.tier ? b.caps1.nc : 0;
      o[7] = b.tier ? (int32_t)b.lds1 : 0;
    }
  return n;
}

extern "C" size_t ostrich_tape_bytes(const ostrich_ctx* ctx) { return ctx ? ctx->tape_total * sizeof(double) : 0; }

// Run f(bucket, stream, tier_ok) for every bucket: on the caller's stream when
// there is one bucket, else each on its own stream between a fork and a join
// event, so that the buckets' launches overlap on the device.  tier_ok says
// whether a tiered bucket may fork once more onto its side stream: not when
// the buckets' streams are themselves forked inside a graph capture (a second
// level of forks under capture has ended the capture with a host crash in the
// HIP runtime; tiered and untiered launches give the same bits, so the graph
// takes the untiered launch).
template <class F> static int for_buckets(ostrich_ctx* ctx, hipStream_t st, F f) {
  if (ctx->buckets.size() == 1) {
    f(ctx->buckets[0], st, true);
    return 0;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_OK(hipStreamIsCapturing(st, &cs));
  const bool tier_ok = cs == hipStreamCaptureStatusNone;
  HIP_OK(hipEventRecord(ctx->ev_fork, st));
  for (size_t i = 0; i < ctx->buckets.size(); ++i) {
    HIP_OK(hipStreamWaitEvent(ctx->bstreams[i], ctx->ev_fork, 0));
    f(ctx->buckets[i], ctx->bstreams[i], tier_ok);
    HIP_OK(hipEventRecord(ctx->ev_join[i], ctx->bstreams[i]));
  }
  for (size_t i = 0; i < ctx->buckets.size(); ++i) HIP_OK(hipStreamWaitEvent(st, ctx->ev_join[i], 0));
  return 0;
}

// The forward kernel of a bucket (team kind by the storage split).  Only the
// banded-LU Newton step is instantiated for the GPU: the matrix-free Krylov
// step is rejected at context creation.
template <class TL, class TG> static decltype(&k_forward<TL, false>) forward_kernel(const Bucket& bk) {
  return bk.split == ost::SPLIT_GLOBAL ? k_forward<TG, false> : k_forward<TL, false>;
}

// One bucket's forward step.  A planning kernel orders the bucket's worlds by
// their estimated cost, most expensive first.  Untiered: one launch over that
// order.  Tiered: the worlds whose contacts exceed the first carve's run with
// the full carve, beside the launch of the others with the first carve on the
// bucket's side stream; that one defers any world it finds too large, and a
// last launch, after both, takes the deferred worlds.
// The worlds of the step are the list wl of n worlds (the bucket's, or a
// caller's list of the context's worlds with the context-wide bucket).
template <class TL, class TG>
static void launch_forward_t(ostrich_ctx* ctx, const Bucket& bk, hipStream_t st, const double* q_prev,
                             const double* u_prev, const double* lam_prev, const double* ctrl, double* q_next,
                             double* u_next, double* lam_next, int32_t* act_slot, int32_t* n_act, int32_t* status,
                             int32_t* iters, double* resnorm, double* tape, const Scratch& sc, const int32_t* wl,
                             int n, bool tier_ok) {
  const int64_t* toff = ctx->d_tape_off;
  const int grid2 = std::min(bk.grid2, n);
  const bool tier = bk.tier && tier_ok;
  int32_t* nact_now = tier ? sc.plan + 2 + 2 * n : nullptr;  // the split by this step's contacts
  if (nact_now)
    hipLaunchKernelGGL(k_count_active, dim3(n), dim3(64), 0, st, ctx->B, ctx->P, wl, q_prev, u_prev,
                       (const int32_t*)ctx->d_hist, nact_now);
  hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, st, ctx->B, wl, n,
                     (const int32_t*)ctx->d_hist, (const int32_t*)nact_now, (const double*)nullptr,
                     (const int64_t*)nullptr, tier ? bk.caps1.nc : 0, sc.plan);
  const int32_t* first = sc.plan + 2;
  const int32_t* second = sc.plan + 2 + n;
  if (tier) {  // the deferral count starts at zero (a fill kernel, also under graph capture)
    hipLaunchKernelGGL(k_zero_i, dim3(1), dim3(64), 0, st, sc.defer, 1);
    (void)hipEventRecord(bk.ev_fork, st);
    (void)hipStreamWaitEvent(bk.side, bk.ev_fork, 0);
    // The full carve's launch stays on the caller's stream and the first carve's
    // goes to the side stream, behind its wait for the fork: so the few large
    // workgroups reach the dispatcher first and find room, instead of waiting
    // for the many small ones to leave a CU with enough free LDS.
    hipLaunchKernelGGL((k_forward<TL, false, true>), dim3(grid2), dim3(bk.team), bk.lds, st, ctx->B, ctx->P,
                       bk.caps, Launch{second, 0, ost::SPLIT_LDS, nullptr, 0, sc.plan + 1, nullptr, ctx->d_hist},
                       q_prev, u_prev, lam_prev, ctrl, q_next, u_next, lam_next, act_slot, n_act, status, iters,
                       resnorm, tape, toff);
    hipLaunchKernelGGL((k_forward<TL, false, false>), dim3(n), dim3(bk.team), bk.lds1, bk.side, ctx->B, ctx->P,
                       bk.caps1, Launch{first, 0, ost::SPLIT_LDS, nullptr, 0, sc.plan, sc.defer, ctx->d_hist}, q_prev,
                       u_prev, lam_prev, ctrl, q_next, u_next, lam_next, act_slot, n_act, status, iters, resnorm, tape,
                       toff);
    (void)hipEventRecord(bk.ev_join, bk.side);
    (void)hipStreamWaitEvent(st, bk.ev_join, 0);
    hipLaunchKernelGGL((k_forward<TL, false, true>), dim3(grid2), dim3(bk.team), bk.lds, st, ctx->B, ctx->P,
                       bk.caps, Launch{sc.defer + 1, 0, ost::SPLIT_LDS, nullptr, 0, sc.defer, nullptr, ctx->d_hist},
                       q_prev, u_prev, lam_prev, ctrl, q_next, u_next, lam_next, act_slot, n_act, status, iters,
                       resnorm, tape, toff);
    return;
  }
  Launch L{first, n, bk.split, bk.split == ost::SPLIT_GLOBAL ? sc.gscr : nullptr, bk.gstride, nullptr, nullptr,
           ctx->d_hist};
  const int grid = bk.split == ost::SPLIT_GLOBAL ? std::max(1, std::min(n, sc.slots)) : n;
  hipLaunchKernelGGL((forward_kernel<TL, TG>(bk)), dim3(grid), dim3(bk.team), bk.lds, st, ctx->B, ctx->P, bk.caps, L,
                     q_prev, u_prev, lam_prev, ctrl, q_next, u_next, lam_next, act_slot, n_act, status, iters, resnorm,
                     tape, toff);
}
// The kernels of the context's batch: with the rim-circle terms compiled in
// only when the batch has rim-circle slots.
static void launch_forward(ostrich_ctx* ctx, const Bucket& bk, hipStream_t st, const double* q_prev,
                           const double* u_prev, const double* lam_prev, const double* ctrl, double* q_next,
                           double* u_next, double* lam_next, int32_t* act_slot, int32_t* n_act, int32_t* status,
                           int32_t* iters, double* resnorm, double* tape, const Scratch& sc, const int32_t* wl,
                           int n, bool tier_ok) {
  if (ctx->rim)
    launch_forward_t<GpuTeamRim, GpuTeamGRim>(ctx, bk, st, q_prev, u_prev, lam_prev, ctrl, q_next, u_next, lam_next,
                                              act_slot, n_act, status, iters, resnorm, tape, sc, wl, n, tier_ok);
  else
    launch_forward_t<GpuTeam, GpuTeamG>(ctx, bk, st, q_prev, u_prev, lam_prev, ctrl, q_next, u_next, lam_next,
                                        act_slot, n_act, status, iters, resnorm, tape, sc, wl, n, tier_ok);
}
static void launch_forward(ostrich_ctx* ctx, const Bucket& bk, hipStream_t st, const double* q_prev,
                           const double* u_prev, const double* lam_prev, const double* ctrl, double* q_next,
                           double* u_next, double* lam_next, int32_t* act_slot, int32_t* n_act, int32_t* status,
                           int32_t* iters, double* resnorm, double* tape, const Scratch& sc, bool tier_ok) {
  launch_forward(ctx, bk, st, q_prev, u_prev, lam_prev, ctrl, q_next, u_next, lam_next, act_slot, n_act, status,
                 iters, resnorm, tape, sc, bk.d_worlds, (int)bk.worlds.size(), tier_ok);
}
static void launch_forward(ostrich_ctx* ctx, const Bucket& bk, hipStream_t st, const double* q_prev,
                           const double* u_prev, const double* lam_prev, const double* ctrl, double* q_next,
                           double* u_next, double* lam_next, int32_t* act_slot, int32_t* n_act, int32_t* status,
                           int32_t* iters, double* resnorm, double* tape, bool tier_ok) {
  launch_forward(ctx, bk, st, q_prev, u_prev, lam_prev, ctrl, q_next, u_next, lam_next, act_slot, n_act, status,
                 iters, resnorm, tape, own_scratch(bk), tier_ok);
}

extern "C" int ostrich_step_forward(ostrich_ctx* ctx, const double* q_prev, const double* u_prev,
                                    const double* lam_prev, const double* ctrl, double* q_next, double* u_next,
                                    double* lam_next, int32_t* act_slot, int32_t* n_act, int32_t* status,
                                    int32_t* iters, double* resnorm, void* tape, void* stream) {
  if (!ctx || !q_prev || !u_prev || !lam_prev || !q_next || !u_next || !lam_next)
    return fail(OSTRICH_E_ARG, "null state pointer");
  if (ctx->NCTRL > 0 && !ctrl) return fail(OSTRICH_E_ARG, "controls required");
  const bool timed = ctx->timing && n_act && iters;
  if (timed) {
    if (ctx->n_ev + 2 > ctx->ev.size()) {
      for (int k = 0; k < 2; ++k) {
        hipEvent_t e;
        HIP_OK(hipEventCreate(&e));
        ctx->ev.push_back(e);
      }
    }
    HIP_OK(hipEventRecord(ctx->ev[ctx->n_ev], (hipStream_t)stream));
  }
  int rc = for_buckets(ctx, (hipStream_t)stream, [&](const Bucket& bk, hipStream_t s, bool tier_ok) {
    launch_forward(ctx, bk, s, q_prev, u_prev, lam_prev, ctrl, q_next, u_next, lam_next, act_slot, n_act, status,
                   iters, resnorm, (double*)tape, tier_ok);
  });
  if (rc) return rc;
  if (timed) {
    HIP_OK(hipEventRecord(ctx->ev[ctx->n_ev + 1], (hipStream_t)stream));
    ctx->n_ev += 2;
    hipLaunchKernelGGL(k_flops, dim3(1), dim3(256), 0, (hipStream_t)stream, ctx->B, n_act, iters, tape ? 1 : 0,
                       ctx->d_flops);
  }
  HIP_OK(hipGetLastError());
  return 0;
}

// ostrich_step_forward with the launches' scratch (deferral queues of tiered
// buckets, slices of buckets kept in device memory) in the static array: no
// allocation, no timing.  A bucket kept in device memory gets as many
// persistent workgroups as its slices that fit, at least one.
extern "C" int ostrich_step_forward_noalloc(ostrich_ctx* ctx, const double* q_prev, const double* u_prev,
                                            const double* lam_prev, const double* ctrl, double* q_next,
                                            double* u_next, double* lam_next, int32_t* act_slot, int32_t* n_act,
                                            int32_t* status, int32_t* iters, double* resnorm, void* tape,
                                            void* stream) {
  if (!ctx || !q_prev || !u_prev || !lam_prev || !q_next || !u_next || !lam_next)
    return fail(OSTRICH_E_ARG, "null state pointer");
  if (ctx->NCTRL > 0 && !ctrl) return fail(OSTRICH_E_ARG, "controls required");
  constexpr int kMaxBuckets = 16;
  if ((int)ctx->buckets.size() > kMaxBuckets) return fail(OSTRICH_E_UNSUPPORTED, "too many buckets");
  char* base = nullptr;
  if (int rc = scratch_dev(&base)) return rc;
  Scratch sc[kMaxBuckets];
  size_t off = 0;
  for (size_t i = 0; i < ctx->buckets.size(); ++i) {
    const Bucket& bk = ctx->buckets[i];
    sc[i] = Scratch{nullptr, nullptr, 0, nullptr};
    {  // the launch plan
      const size_t n = al256((3 * bk.worlds.size() + 2) * sizeof(int32_t));
      if (off + n > kScratchBytes)
        return fail(OSTRICH_E_WORKSPACE, "the batch needs more than the " + std::to_string(kScratchBytes >> 20) +
                                             " MiB of static scratch");
      sc[i].plan = (int32_t*)(base + off);
      off += n;
    }
    if (bk.tier) {
      const size_t n = al256((bk.worlds.size() + 1) * sizeof(int32_t));
      if (off + n > kScratchBytes)
        return fail(OSTRICH_E_WORKSPACE, "the batch needs more than the " + std::to_string(kScratchBytes >> 20) +
                                             " MiB of static scratch");
      sc[i].defer = (int32_t*)(base + off);
      off += n;
    }
    if (bk.split == ost::SPLIT_GLOBAL) {
      const size_t per = bk.gstride * sizeof(double);
      const size_t fit = off < kScratchBytes ? (kScratchBytes - off) / per : 0;
      const int slots = (int)std::min<size_t>(std::max(bk.slots, 1), fit);
      if (slots < 1)
        return fail(OSTRICH_E_WORKSPACE, "a world kept in device memory needs more than the " +
                                             std::to_string(kScratchBytes >> 20) + " MiB of static scratch");
      sc[i].gscr = (double*)(base + off);
      sc[i].slots = slots;
      off += al256((size_t)slots * per);
    }
  }
  int rc = for_buckets(ctx, (hipStream_t)stream, [&](const Bucket& bk, hipStream_t s, bool tier_ok) {
    launch_forward(ctx, bk, s, q_prev, u_prev, lam_prev, ctrl, q_next, u_next, lam_next, act_slot, n_act, status,
                   iters, resnorm, (double*)tape, sc[&bk - ctx->buckets.data()], tier_ok);
  });
  if (rc) return rc;
  HIP_OK(hipGetLastError());
  return 0;
}

extern "C" int ostrich_ctx_timing(ostrich_ctx* ctx, int32_t mode, double* out) {
  if (!ctx) return fail(OSTRICH_E_ARG, "null context");
  if (mode == 1 || mode == 0) {  // start (reset) or stop
    if (!ctx->d_flops) HIP_OK(ctx_malloc(ctx, &ctx->d_flops, 4 * sizeof(double)));
    if (mode == 1) {
      HIP_OK(hipDeviceSynchronize());
      const double z[4] = {0.0, 0.0, 0.0, 0.0};
      HIP_OK(hipMemcpy(ctx->d_flops, z, sizeof(z), hipMemcpyHostToDevice));
      ctx->n_ev = 0;
      ctx->n_eva = 0;
    }
    ctx->timing = mode == 1;
    return 0;
  }
  if ((mode != 2 && mode != 3) || !out) return fail(OSTRICH_E_ARG, "timing mode");
  if (!ctx->d_flops) {
    out[0] = out[1] = out[2] = out[3] = 0.0;
    return 0;
  }
  HIP_OK(hipDeviceSynchronize());
  const std::vector<hipEvent_t>& ev = mode == 2 ? ctx->ev : ctx->eva;
  const size_t n_ev = mode == 2 ? ctx->n_ev : ctx->n_eva;
  double total = 0.0;
  for (size_t i = 0; i + 1 < n_ev; i += 2) {
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
    total += ms;
  }
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  HIP_OK(hipMemcpy(acc, ctx->d_flops, sizeof(acc), hipMemcpyDeviceToHost));
  out[0] = (double)(n_ev / 2);
  out[1] = total;
  out[2] = acc[mode - 2];
  out[3] = acc[mode];
  return 0;
}

// One bucket's adjoint step over the list wl of n worlds, as the forward
// (launch_forward): the plan's estimates and the first carve's split come from
// the row counts the tape records, which are this step's.
template <class TL, class TG>
static void launch_adjoint_t(ostrich_ctx* ctx, const Bucket& bk, hipStream_t s, const int32_t* wl, int n,
                             const double* q_prev, const double* u_prev, const double* ctrl, const double* u_next,
                             const double* lam_next, const double* tp, const double* gq_next, const double* gu_next,
                             double* gq_prev, double* gu_prev, double* g_ctrl, int rf, double* g_mass, double* g_mu,
                             double* g_kp, int32_t* adj_status, bool tier_ok) {
  const int64_t* toff = ctx->d_tape_off;
  const int grid2 = std::min(bk.grid2, n);
  const bool tier = bk.tier && tier_ok;
  hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, s, ctx->B, wl, n, (const int32_t*)nullptr,
                     (const int32_t*)nullptr, tp, toff, tier ? bk.caps1.nc : 0, bk.d_plan);
  const int32_t* first = bk.d_plan + 2;
  const int32_t* second = bk.d_plan + 2 + n;
  if (tier) {
    hipLaunchKernelGGL(k_zero_i, dim3(1), dim3(64), 0, s, bk.d_defer, 1);
    (void)hipEventRecord(bk.ev_fork, s);
    (void)hipStreamWaitEvent(bk.side, bk.ev_fork, 0);
    hipLaunchKernelGGL((k_adjoint<TL, true>), dim3(grid2), dim3(bk.team), bk.lds_adj, s, ctx->B, ctx->P,
                       bk.caps, Launch{second, 0, ost::SPLIT_LDS, nullptr, 0, bk.d_plan + 1, nullptr, nullptr}, q_prev,
                       u_prev, ctrl, u_next, lam_next, tp, toff, gq_next, gu_next, gq_prev, gu_prev, g_ctrl, rf,
                       g_mass, g_mu, g_kp, adj_status);
    hipLaunchKernelGGL((k_adjoint<TL, false>), dim3(n), dim3(bk.team), bk.lds1_adj, bk.side, ctx->B, ctx->P,
                       bk.caps1, Launch{first, 0, ost::SPLIT_LDS, nullptr, 0, bk.d_plan, bk.d_defer, nullptr}, q_prev,
                       u_prev, ctrl, u_next, lam_next, tp, toff, gq_next, gu_next, gq_prev, gu_prev, g_ctrl, rf, g_mass,
                       g_mu, g_kp, adj_status);
    (void)hipEventRecord(bk.ev_join, bk.side);
    (void)hipStreamWaitEvent(s, bk.ev_join, 0);
    hipLaunchKernelGGL((k_adjoint<TL, true>), dim3(grid2), dim3(bk.team), bk.lds_adj, s, ctx->B, ctx->P,
                       bk.caps, Launch{bk.d_defer + 1, 0, ost::SPLIT_LDS, nullptr, 0, bk.d_defer, nullptr, nullptr},
                       q_prev, u_prev, ctrl, u_next, lam_next, tp, toff, gq_next, gu_next, gq_prev, gu_prev, g_ctrl,
                       rf, g_mass, g_mu, g_kp, adj_status);
    return;
  }
  Launch L{first, n, bk.split, bk.split == ost::SPLIT_GLOBAL ? bk.gscr : nullptr, bk.gstride, nullptr, nullptr,
           nullptr};
  const int grid = bk.split == ost::SPLIT_GLOBAL ? std::max(1, std::min(n, bk.slots)) : n;
  hipLaunchKernelGGL(bk.split == ost::SPLIT_GLOBAL ? k_adjoint<TG> : k_adjoint<TL>, dim3(grid),
                     dim3(bk.team), bk.lds_adj, s, ctx->B, ctx->P, bk.caps, L, q_prev, u_prev, ctrl, u_next, lam_next,
                     tp, toff, gq_next, gu_next, gq_prev, gu_prev, g_ctrl, rf, g_mass, g_mu, g_kp, adj_status);
}
static void launch_adjoint(ostrich_ctx* ctx, const Bucket& bk, hipStream_t s, const int32_t* wl, int n,
                           const double* q_prev, const double* u_prev, const double* ctrl, const double* u_next,
                           const double* lam_next, const double* tp, const double* gq_next, const double* gu_next,
                           double* gq_prev, double* gu_prev, double* g_ctrl, int rf, double* g_mass, double* g_mu,
                           double* g_kp, int32_t* adj_status, bool tier_ok) {
  if (ctx->rim)
    launch_adjoint_t<GpuTeamRim, GpuTeamGRim>(ctx, bk, s, wl, n, q_prev, u_prev, ctrl, u_next, lam_next, tp, gq_next,
                                              gu_next, gq_prev, gu_prev, g_ctrl, rf, g_mass, g_mu, g_kp, adj_status,
                                              tier_ok);
  else
    launch_adjoint_t<GpuTeam, GpuTeamG>(ctx, bk, s, wl, n, q_prev, u_prev, ctrl, u_next, lam_next, tp, gq_next,
                                        gu_next, gq_prev, gu_prev, g_ctrl, rf, g_mass, g_mu, g_kp, adj_status,
                                        tier_ok);
}

static int adjoint_step(ostrich_ctx* ctx, const double* q_prev, const double* u_prev, const double* ctrl,
                        const double* u_next, const double* lam_next, const void* tape, const double* gq_next,
                        const double* gu_next, double* gq_prev, double* gu_prev, double* g_ctrl, double* g_mass,
                        double* g_mu, double* g_kp, int32_t refine, int32_t* adj_status, void* stream) {
  if (!ctx || !q_prev || !u_prev || !u_next || !lam_next || !tape || !gq_next || !gu_next || !gq_prev || !gu_prev)
    return fail(OSTRICH_E_ARG, "null pointer");
  if (ctx->NCTRL > 0 && (!ctrl || !g_ctrl)) return fail(OSTRICH_E_ARG, "controls required");
  int rf = refine < 0 ? ctx->refine : refine;
  const bool timed = ctx->timing && ctx->d_flops;
  if (timed) {
    if (ctx->n_eva + 2 > ctx->eva.size()) {
      for (int k = 0; k < 2; ++k) {
        hipEvent_t e;
        HIP_OK(hipEventCreate(&e));
        ctx->eva.push_back(e);
      }
    }
    HIP_OK(hipEventRecord(ctx->eva[ctx->n_eva], (hipStream_t)stream));
  }
  int rc = for_buckets(ctx, (hipStream_t)stream, [&](const Bucket& bk, hipStream_t s, bool tier_ok) {
    launch_adjoint(ctx, bk, s, bk.d_worlds, (int)bk.worlds.size(), q_prev, u_prev, ctrl, u_next, lam_next,
                   (const double*)tape, gq_next, gu_next, gq_prev, gu_prev, g_ctrl, rf, g_mass, g_mu, g_kp,
                   adj_status, tier_ok);
  });
  if (rc) return rc;
  if (timed) {
    HIP_OK(hipEventRecord(ctx->eva[ctx->n_eva + 1], (hipStream_t)stream));
    ctx->n_eva += 2;
    hipLaunchKernelGGL(k_abytes, dim3(1), dim3(256), 0, (hipStream_t)stream, ctx->B, (const double*)tape,
                       (const int64_t*)ctx->d_tape_off, ctx->d_flops);
  }
  HIP_OK(hipGetLastError());
  return 0;
}

extern "C" int ostrich_step_adjoint(ostrich_ctx* ctx, const double* q_prev, const double* u_prev,
                                    const double* ctrl, const double* u_next, const double* lam_next,
                                    const void* tape, const double* gq_next, const double* gu_next, double* gq_prev,
                                    double* gu_prev, double* g_ctrl, int32_t refine, int32_t* adj_status,
                                    void* stream) {
  return adjoint_step(ctx, q_prev, u_prev, ctrl, u_next, lam_next, tape, gq_next, gu_next, gq_prev, gu_prev, g_ctrl,
                      nullptr, nullptr, nullptr, refine, adj_status, stream);
}

extern "C" int ostrich_step_adjoint_params(ostrich_ctx* ctx, const double* q_prev, const double* u_prev,
                                           const double* ctrl, const double* u_next, const double* lam_next,
                                           const void* tape, const double* gq_next, const double* gu_next,
                                           double* gq_prev, double* gu_prev, double* g_ctrl, double* g_mass,
                                           double* g_mu, double* g_kp, int32_t refine, int32_t* adj_status,
                                           void* stream) {
  if (!g_mass || !g_mu || !g_kp) return fail(OSTRICH_E_ARG, "parameter cotangent outputs required");
  return adjoint_step(ctx, q_prev, u_prev, ctrl, u_next, lam_next, tape, gq_next, gu_next, gq_prev, gu_prev, g_ctrl,
                      g_mass, g_mu, g_kp, refine, adj_status, stream);
}

static Launch list_launch(const ostrich_ctx* ctx, const int32_t* worlds, int n) {
  return Launch{worlds, n, ctx->all.split, ctx->all.split == ost::SPLIT_GLOBAL ? ctx->all.gscr : nullptr,
                ctx->all.gstride};
}
static int list_grid(const ostrich_ctx* ctx, int n) {
  return ctx->all.split == ost::SPLIT_GLOBAL ? std::max(1, std::min(n, ctx->all.slots)) : n;
}

extern "C" int ostrich_step_forward_list(ostrich_ctx* ctx, const int32_t* worlds, int32_t n, const double* q_prev,
                                         const double* u_prev, const double* lam_prev, const double* ctrl,
                                         double* q_next, double* u_next, double* lam_next, int32_t* act_slot,
                                         int32_t* n_act, int32_t* status, int32_t* iters, double* resnorm,
                                         void* tape, void* stream) {
  if (!ctx || !worlds || n < 0 || n > ctx->W) return fail(OSTRICH_E_ARG, "world list");
  if (!q_prev || !u_prev || !lam_prev || !q_next || !u_next || !lam_next)
    return fail(OSTRICH_E_ARG, "null state pointer");
  if (ctx->NCTRL > 0 && !ctrl) return fail(OSTRICH_E_ARG, "controls required");
  if (n == 0) return 0;
  launch_forward(ctx, ctx->all, (hipStream_t)stream, q_prev, u_prev, lam_prev, ctrl, q_next, u_next, lam_next,
                 act_slot, n_act, status, iters, resnorm, (double*)tape, own_scratch(ctx->all), worlds, n, true);
  HIP_OK(hipGetLastError());
  return 0;
}

extern "C" int ostrich_step_adjoint_list(ostrich_ctx* ctx, const int32_t* worlds, int32_t n, const double* q_prev,
                                         const double* u_prev, const double* ctrl, const double* u_next,
                                         const double* lam_next, const void* tape, const double* gq_next,
                                         const double* gu_next, double* gq_prev, double* gu_prev, double* g_ctrl,
                                         int32_t refine, int32_t* adj_status, void* stream) {
  if (!ctx || !worlds || n < 0 || n > ctx->W) return fail(OSTRICH_E_ARG, "world list");
  if (!q_prev || !u_prev || !u_next || !lam_next || !tape || !gq_next || !gu_next || !gq_prev || !gu_prev)
    return fail(OSTRICH_E_ARG, "null pointer");
  if (ctx->NCTRL > 0 && (!ctrl || !g_ctrl)) return fail(OSTRICH_E_ARG, "controls required");
  if (n == 0) return 0;
  const int rf = refine < 0 ? ctx->refine : refine;
  launch_adjoint(ctx, ctx->all, (hipStream_t)stream, worlds, n, q_prev, u_prev, ctrl, u_next, lam_next,
                 (const double*)tape, gq_next, gu_next, gq_prev, gu_prev, g_ctrl, rf, nullptr, nullptr, nullptr,
                 adj_status, true);
  HIP_OK(hipGetLastError());
  return 0;
}

extern "C" int ostrich_step_forward_plain(ostrich_ctx* ctx, const double* q_prev, const double* u_prev,
                                          const double* lam_prev, const double* ctrl, double* q_next,
                                          double* u_next, double* lam_next, int32_t* act_slot, int32_t* n_act,
                                          int32_t* status, int32_t* iters, double* resnorm, void* tape,
                                          void* stream) {
  if (!ctx || !q_prev || !u_prev || !lam_prev || !q_next || !u_next || !lam_next)
    return fail(OSTRICH_E_ARG, "null state pointer");
  if (ctx->NCTRL > 0 && !ctrl) return fail(OSTRICH_E_ARG, "controls required");
  if (ctx->P.lin != OSTRICH_LIN_LU) return fail(OSTRICH_E_UNSUPPORTED, "the plain path steps with the banded LU");
  hipStream_t st = (hipStream_t)stream;
  const size_t lds = 0;
  for (int w = 0; w < ctx->W; ++w) {
    hipLaunchKernelGGL(k_plain_begin, dim3(1), dim3(kPlainTeam), lds, st, ctx->B, ctx->P, ctx->caps, w, q_prev,
                       u_prev, lam_prev, ctrl, ctx->plain_ws);
    for (int k = 1; k <= ctx->P.kmax; ++k)
      hipLaunchKernelGGL(k_plain_iteration, dim3(1), dim3(kPlainTeam), lds, st, ctx->B, ctx->P, ctx->caps, w, ctrl,
                         ctx->plain_ws, k);
    hipLaunchKernelGGL(k_plain_end, dim3(1), dim3(kPlainTeam), lds, st, ctx->B, ctx->P, ctx->caps, w, ctrl, q_next,
                       u_next, lam_next, act_slot, n_act, status, iters, resnorm, (double*)tape,
                       (const int64_t*)ctx->d_tape_off, ctx->plain_ws);
  }
  HIP_OK(hipGetLastError());
  return 0;
}

extern "C" int ostrich_step_adjoint_plain(ostrich_ctx* ctx, const double* q_prev, const double* u_prev,
                                          const double* ctrl, const double* u_next, const double* lam_next,
                                          const void* tape, const double* gq_next, const double* gu_next,
                                          double* gq_prev, double* gu_prev, double* g_ctrl, int32_t refine,
                                          int32_t* adj_status, void* stream) {
  if (!ctx || !q_prev || !u_prev || !u_next || !lam_next || !tape || !gq_next || !gu_next || !gq_prev || !gu_prev)
    return fail(OSTRICH_E_ARG, "null pointer");
  if (ctx->NCTRL > 0 && (!ctrl || !g_ctrl)) return fail(OSTRICH_E_ARG, "controls required");
  int rf = refine < 0 ? ctx->refine : refine;
  const Bucket& bk = ctx->all;
  if (!bk.d_worlds || (int)bk.worlds.size() != ctx->W) return fail(OSTRICH_E_ARG, "context world list missing");
  for (int w = 0; w < ctx->W; ++w)  // one launch per world, over the one-world list {w}
    hipLaunchKernelGGL(ctx->rim ? (bk.split == ost::SPLIT_GLOBAL ? k_adjoint<GpuTeamGRim> : k_adjoint<GpuTeamRim>)
                                : (bk.split == ost::SPLIT_GLOBAL ? k_adjoint<GpuTeamG> : k_adjoint<GpuTeam>),
                       dim3(1),
                       dim3(bk.team), bk.lds_adj, (hipStream_t)stream, ctx->B, ctx->P, bk.caps,
                       list_launch(ctx, bk.d_worlds + w, 1), q_prev, u_prev, ctrl, u_next, lam_next,
                       (const double*)tape, (const int64_t*)ctx->d_tape_off, gq_next, gu_next, gq_prev, gu_prev,
                       g_ctrl, rf, (double*)nullptr, (double*)nullptr, (double*)nullptr, adj_status);
  HIP_OK(hipGetLastError());
  return 0;
}

// Autotuner: for every bucket, time one forward step of its worlds under each
// candidate launch (team 64 / 128 / 256, Schur matrix on chip or in device
// memory) and keep the fastest.  The per-world arithmetic is the same under
// every candidate, so the choice changes only the time.
extern "C" int ostrich_autotune(ostrich_ctx* ctx, const double* q, const double* u, const double* lam,
                                const double* ctrl, int32_t reps, void* stream) {
  if (!ctx || !q || !u || !lam) return fail(OSTRICH_E_ARG, "null argument");
  if (ctx->NCTRL > 0 && !ctrl) return fail(OSTRICH_E_ARG, "controls required");
  if (reps < 1) reps = 1;
  hipStream_t st = (hipStream_t)stream;
  const int W = ctx->W, NB = ctx->NB;
  double *qn = nullptr, *un = nullptr, *ln = nullptr, *rn = nullptr;
  int32_t *as = nullptr, *na = nullptr, *ss = nullptr, *it = nullptr;
  auto cleanup = [&]() {
    for (void* p : {(void*)qn, (void*)un, (void*)ln, (void*)rn, (void*)as, (void*)na, (void*)ss, (void*)it})
      if (p) (void)hipFree(p);
  };
  hipEvent_t e0, e1;
  int rc = 0;
  if (hipMalloc(&qn, sizeof(double) * 7 * NB) || hipMalloc(&un, sizeof(double) * 6 * NB) ||
      hipMalloc(&ln, sizeof(double) * std::max(ctx->NL, 1)) || hipMalloc(&rn, sizeof(double) * W) ||
      hipMalloc(&as, sizeof(int32_t) * std::max(ctx->NS, 1)) || hipMalloc(&na, sizeof(int32_t) * W) ||
      hipMalloc(&ss, sizeof(int32_t) * W) || hipMalloc(&it, sizeof(int32_t) * W)) {
    cleanup();
    return fail(OSTRICH_E_HIP, "autotune scratch allocation failed");
  }
  if (hipEventCreate(&e0) || hipEventCreate(&e1)) {
    cleanup();
    return fail(OSTRICH_E_HIP, "hipEventCreate failed");
  }
  for (Bucket& bk : ctx->buckets) {
    float best = 1e30f;
    int bt = bk.team, bs = bk.split;
    bool btier = bk.tier;
    struct Cand { int split, team; bool tier; };
    std::vector<Cand> cands;
    for (int split : {ost::SPLIT_LDS, ost::SPLIT_GLOBAL})
      for (int team : {64, 128, 256})
        for (bool tier : {true, false})
          if (ost::world_lds_bytes(bk.caps, team, split, true) <= ctx->lds_limit &&
              (split == ost::SPLIT_LDS || !tier))
            cands.push_back(Cand{split, team, tier});
    for (const Cand& cd : cands) {
      if ((rc = configure_bucket(ctx, bk, cd.team, cd.split, cd.tier))) break;
      if (cd.tier && !bk.tier) continue;  // no tiered carve for this team: its untiered candidate follows
      launch_forward(ctx, bk, st, q, u, lam, ctrl, qn, un, ln, as, na, ss, it, rn, nullptr, true);  // warm
      (void)hipEventRecord(e0, st);
      for (int r = 0; r < reps; ++r)
        launch_forward(ctx, bk, st, q, u, lam, ctrl, qn, un, ln, as, na, ss, it, rn, nullptr, true);
      (void)hipEventRecord(e1, st);
      if (hipEventSynchronize(e1) != hipSuccess || hipGetLastError() != hipSuccess) {
        rc = fail(OSTRICH_E_HIP, "autotune launch failed");
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms < best) { best = ms; bt = cd.team; bs = cd.split; btier = bk.tier; }
    }
    if (rc) break;
    if ((rc = configure_bucket(ctx, bk, bt, bs, btier))) break;
    bk.tuned = true;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  cleanup();
  return rc;
}

// ------------------------------------------------------------------ rollout
namespace {
struct RollLayout {
  size_t S, tape, ctrl, ck_states, seg_states, seg_tapes, grads, ints, total;
  int n_seg;
};
inline size_t al(size_t x) { return (x + 31) & ~size_t(31); }

RollLayout roll_layout(const ostrich_ctx* c, int T, int ck) {
  RollLayout L;
  L.S = (size_t)7 * c->NB + 6 * c->NB + c->NL;
  L.tape = c->tape_total;
  L.ctrl = al((size_t)T * std::max(c->NCTRL, 1));
  if (ck <= 0) {
    L.n_seg = 0;
    L.ck_states = (size_t)(T + 1) * L.S;
    L.seg_states = 0;
    L.seg_tapes = (size_t)T * L.tape;
  } else {
    L.n_seg = (T + ck - 1) / ck;
    L.ck_states = (size_t)L.n_seg * L.S + 2 * L.S;  // checkpoints + forward ping-pong
    L.seg_states = (size_t)(ck + 1) * L.S;
    L.seg_tapes = (size_t)ck * L.tape;
  }
  L.grads = al((size_t)2 * 7 * c->NB + 2 * 6 * c->NB + std::max(c->NCTRL, 1) + c->W);
  L.ints = al((size_t)c->NS + 3 * c->W + 8);
  L.total = (L.ctrl + al(L.ck_states) + al(L.seg_states) + al(L.seg_tapes) + L.grads) * sizeof(double) +
            L.ints * sizeof(int32_t);
  return L;
}
}  // namespace

extern "C" size_t ostrich_rollout_workspace_bytes(const ostrich_ctx* ctx, int32_t T, int32_t ckpt_every) {
  if (!ctx || T < 1) return 0;
  return roll_layout(ctx, T, ckpt_every).total;
}

// Rollout with the final-xy loss (spec == nullptr, target [W*2]) or the shaped
// loss of `spec` (target unused).
static int rollout_run(ostrich_ctx* ctx, int32_t phase, const double* q0, const double* u0, const double* knots,
                       int32_t K, const double* basis, int32_t T, int32_t ckpt_every, const int32_t* loss_body,
                       const double* target, const ostrich_loss* spec, const double* loss_grad, double* loss,
                       double* qT, double* uT, double* g_q0, double* g_u0, double* g_knots, void* workspace,
                       size_t workspace_bytes, int32_t* status_or, void* stream_) {
  if (!ctx || !q0 || !u0 || T < 1 || !workspace || !loss_body || (!target && !spec))
    return fail(OSTRICH_E_ARG, "null argument or T < 1");
  LossDev LD{};
  if (spec) {
    LD = LossDev{spec->w_pos, spec->w_head, spec->w_vel, spec->w_ctrl, spec->w_track, spec->w_yaw, spec->goal,
                 spec->ref};
    const double wts[6] = {LD.w_pos, LD.w_head, LD.w_vel, LD.w_ctrl, LD.w_track, LD.w_yaw};
    for (double v : wts)
      if (!std::isfinite(v)) return fail(OSTRICH_E_ARG, "loss weights must be finite");
    if (!LD.goal) return fail(OSTRICH_E_ARG, "loss goal required");
    if ((LD.w_track != 0.0 || LD.w_yaw != 0.0) && !LD.ref) return fail(OSTRICH_E_ARG, "loss reference required");
  }
  const bool per_step = spec && (LD.w_track != 0.0 || LD.w_yaw != 0.0);
  const bool ctrl_reg = spec && LD.w_ctrl != 0.0 && ctx->NCTRL > 0;
  if (ctx->NCTRL > 0 && (!knots || !basis || K < 1)) return fail(OSTRICH_E_ARG, "knots and basis required");
  if (!(phase & (OSTRICH_FORWARD | OSTRICH_BACKWARD))) return fail(OSTRICH_E_ARG, "phase");
  RollLayout L = roll_layout(ctx, T, ckpt_every);
  if (workspace_bytes < L.total) return fail(OSTRICH_E_WORKSPACE, "rollout workspace too small");
  hipStream_t st = (hipStream_t)stream_;
  const int W = ctx->W, NB = ctx->NB, NL = ctx->NL, NC = std::max(ctx->NCTRL, 1);
  double* base = (double*)workspace;
  double* ctrl = base;
  double* ck = ctrl + L.ctrl;
  double* seg = ck + al(L.ck_states);
  double* segt = seg + al(L.seg_states);
  double* gr = segt + al(L.seg_tapes);
  int32_t* ib = (int32_t*)(gr + L.grads);
  double* gqa = gr;
  double* gqb = gqa + 7 * NB;
  double* gua = gqb + 7 * NB;
  double* gub = gua + 6 * NB;
  double* gc = gub + 6 * NB;
  double* resn = gc + NC;
  int32_t* act = ib;
  int32_t* nact = act + ctx->NS;
  int32_t* sts = nact + W;
  int32_t* its = sts + W;
  auto st_q = [&](double* s) { return s; };
  auto st_u = [&](double* s) { return s + 7 * NB; };
  auto st_l = [&](double* s) { return s + 13 * NB; };
  auto tape_at = [&](double* t0, int j) { return t0 + (size_t)j * L.tape; };
  const double* ctrl_k0 = nullptr;
  auto ctrl_at = [&](int k) -> const double* { return ctx->NCTRL > 0 ? ctrl + (size_t)k * ctx->NCTRL : ctrl_k0; };
  int rc;
  if (phase & OSTRICH_FORWARD) {
    if (ctx->NCTRL > 0)
      hipLaunchKernelGGL(k_ctrl, dim3(nblk((long)T * ctx->NCTRL, 256)), dim3(256), 0, st, basis, knots, T, K,
                         ctx->NCTRL, ctrl);
    if (status_or) hipLaunchKernelGGL(k_zero_i, dim3(nblk(W, 256)), dim3(256), 0, st, status_or, W);
    double* s0 = ck;
    HIP_OK(hipMemcpyAsync(st_q(s0), q0, sizeof(double) * 7 * NB, hipMemcpyDeviceToDevice, st));
    HIP_OK(hipMemcpyAsync(st_u(s0), u0, sizeof(double) * 6 * NB, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_fill, dim3(nblk(NL, 256)), dim3(256), 0, st, st_l(s0), (long)NL, 0.0);
    double* cur = s0;
    if (spec && loss) hipLaunchKernelGGL(k_fill, dim3(nblk(W, 256)), dim3(256), 0, st, loss, (long)W, 0.0);
    for (int k = 0; k < T; ++k) {
      double* nxt;
      double* tp = nullptr;
      if (ckpt_every <= 0) {
        nxt = ck + (size_t)(k + 1) * L.S;
        tp = tape_at(segt, k);
      } else {
        nxt = ck + (size_t)L.n_seg * L.S + (size_t)((k + 1) & 1) * L.S;
      }
      rc = ostrich_step_forward(ctx, st_q(cur), st_u(cur), st_l(cur), ctrl_at(k), st_q(nxt), st_u(nxt), st_l(nxt),
                                act, nact, sts, its, resn, tp, st);
      if (rc) return rc;
      if (status_or) hipLaunchKernelGGL(k_or, dim3(nblk(W, 256)), dim3(256), 0, st, status_or, sts, W);
      if (loss && (per_step || (spec && k + 1 == T)))
        hipLaunchKernelGGL(k_state_loss, dim3(nblk(W, 256)), dim3(256), 0, st, ctx->B.body_off, W, st_q(nxt),
                           st_u(nxt), loss_body, LD, k + 1, (int)T, (const double*)nullptr, loss, (double*)nullptr,
                           (double*)nullptr, status_or);
      cur = nxt;
      if (ckpt_every > 0 && (k + 1) % ckpt_every == 0 && k + 1 < T) {
        double* dst = ck + (size_t)((k + 1) / ckpt_every) * L.S;
        HIP_OK(hipMemcpyAsync(dst, cur, sizeof(double) * L.S, hipMemcpyDeviceToDevice, st));
      }
    }
    if (qT) HIP_OK(hipMemcpyAsync(qT, st_q(cur), sizeof(double) * 7 * NB, hipMemcpyDeviceToDevice, st));
    if (uT) HIP_OK(hipMemcpyAsync(uT, st_u(cur), sizeof(double) * 6 * NB, hipMemcpyDeviceToDevice, st));
    // keep the final state where the backward pass finds it
    if (ckpt_every > 0) {
      double* fin = ck + (size_t)L.n_seg * L.S;
      if (cur != fin) HIP_OK(hipMemcpyAsync(fin, cur, sizeof(double) * L.S, hipMemcpyDeviceToDevice, st));
    }
    if (!spec)
      hipLaunchKernelGGL(k_loss, dim3(nblk(W, 256)), dim3(256), 0, st, ctx->B.body_off, W, st_q(cur), loss_body,
                         target, (const double*)nullptr, loss, (double*)nullptr, status_or);
    else if (ctrl_reg && loss)
      hipLaunchKernelGGL(k_ctrl_loss, dim3(nblk(W, 256)), dim3(256), 0, st, ctx->B.ctrl_off, W, ctrl, (int)T,
                         ctx->NCTRL, LD.w_ctrl / T, loss);
  }
  if (phase & OSTRICH_BACKWARD) {
    if (!g_q0 || !g_u0 || (ctx->NCTRL > 0 && !g_knots)) return fail(OSTRICH_E_ARG, "gradient outputs required");
    double* fin = ckpt_every <= 0 ? ck + (size_t)T * L.S : ck + (size_t)L.n_seg * L.S;
    hipLaunchKernelGGL(k_fill, dim3(nblk(7 * NB, 256)), dim3(256), 0, st, gqa, (long)7 * NB, 0.0);
    hipLaunchKernelGGL(k_fill, dim3(nblk(6 * NB, 256)), dim3(256), 0, st, gua, (long)6 * NB, 0.0);
    if (ctx->NCTRL > 0)
      hipLaunchKernelGGL(k_fill, dim3(nblk((long)ctx->NCTRL * K, 256)), dim3(256), 0, st, g_knots,
                         (long)ctx->NCTRL * K, 0.0);
    if (!spec)
      hipLaunchKernelGGL(k_loss, dim3(nblk(W, 256)), dim3(256), 0, st, ctx->B.body_off, W, st_q(fin), loss_body,
                         target, loss_grad, (double*)nullptr, gqa, status_or);
    else
      hipLaunchKernelGGL(k_state_loss, dim3(nblk(W, 256)), dim3(256), 0, st, ctx->B.body_off, W, st_q(fin),
                         st_u(fin), loss_body, LD, (int)T, (int)T, loss_grad, (double*)nullptr, gqa, gua, status_or);
    double *gq = gqa, *gq2 = gqb, *gu = gua, *gu2 = gub;
    // adjoint of step k: cotangents of state k + 1 (its own loss terms included)
    // to those of state k, to which state k's loss terms are then added
    auto adj = [&](double* sm, double* sp, double* tp, int k) -> int {
      int r = ostrich_step_adjoint(ctx, st_q(sm), st_u(sm), ctrl_at(k), st_u(sp), st_l(sp), tp, gq, gu, gq2, gu2,
                                   gc, -1, status_or, st);
      if (r) return r;
      if (ctrl_reg)
        hipLaunchKernelGGL(k_ctrl_reg_grad, dim3(nblk(W, 256)), dim3(256), 0, st, ctx->B.ctrl_off, W, ctrl_at(k),
                           LD.w_ctrl / T, loss_grad, gc);
      if (ctx->NCTRL > 0)
        hipLaunchKernelGGL(k_gknots, dim3(nblk((long)ctx->NCTRL * K, 256)), dim3(256), 0, st, basis, gc, k, K,
                           ctx->NCTRL, g_knots);
      std::swap(gq, gq2);
      std::swap(gu, gu2);
      if (per_step && k >= 1)
        hipLaunchKernelGGL(k_state_loss, dim3(nblk(W, 256)), dim3(256), 0, st, ctx->B.body_off, W, st_q(sm),
                           st_u(sm), loss_body, LD, k, (int)T, loss_grad, (double*)nullptr, gq, gu, status_or);
      return 0;
    };
    if (ckpt_every <= 0) {
      for (int k = T - 1; k >= 0; --k) {
        rc = adj(ck + (size_t)k * L.S, ck + (size_t)(k + 1) * L.S, tape_at(segt, k), k);
        if (rc) return rc;
      }
    } else {
      for (int s = L.n_seg - 1; s >= 0; --s) {
        int k0 = s * ckpt_every, len = std::min(ckpt_every, T - k0);
        HIP_OK(hipMemcpyAsync(seg, ck + (size_t)s * L.S, sizeof(double) * L.S, hipMemcpyDeviceToDevice, st));
        for (int j = 0; j < len; ++j) {  // recompute the segment, storing states and factors
          double* a = seg + (size_t)j * L.S;
          double* b = seg + (size_t)(j + 1) * L.S;
          rc = ostrich_step_forward(ctx, st_q(a), st_u(a), st_l(a), ctrl_at(k0 + j), st_q(b), st_u(b), st_l(b), act,
                                    nact, sts, its, resn, tape_at(segt, j), st);
          if (rc) return rc;
        }
        for (int j = len - 1; j >= 0; --j) {
          rc = adj(seg + (size_t)j * L.S, seg + (size_t)(j + 1) * L.S, tape_at(segt, j), k0 + j);
          if (rc) return rc;
        }
      }
    }
    HIP_OK(hipMemcpyAsync(g_q0, gq, sizeof(double) * 7 * NB, hipMemcpyDeviceToDevice, st));
    HIP_OK(hipMemcpyAsync(g_u0, gu, sizeof(double) * 6 * NB, hipMemcpyDeviceToDevice, st));
  }
  return 0;
}

extern "C" int ostrich_rollout(ostrich_ctx* ctx, int32_t phase, const double* q0, const double* u0,
                               const double* knots, int32_t K, const double* basis, int32_t T, int32_t ckpt_every,
                               const int32_t* loss_body, const double* target, const double* loss_grad,
                               double* loss, double* qT, double* uT, double* g_q0, double* g_u0, double* g_knots,
                               void* workspace, size_t workspace_bytes, int32_t* status_or, void* stream) {
  if (!target) return fail(OSTRICH_E_ARG, "target required");
  return rollout_run(ctx, phase, q0, u0, knots, K, basis, T, ckpt_every, loss_body, target, nullptr, loss_grad, loss,
                     qT, uT, g_q0, g_u0, g_knots, workspace, workspace_bytes, status_or, stream);
}

extern "C" int ostrich_rollout_shaped(ostrich_ctx* ctx, int32_t phase, const double* q0, const double* u0,
                                      const double* knots, int32_t K, const double* basis, int32_t T,
                                      int32_t ckpt_every, const int32_t* loss_body, const ostrich_loss* spec,
                                      const double* loss_grad, double* loss, double* qT, double* uT, double* g_q0,
                                      double* g_u0, double* g_knots, void* workspace, size_t workspace_bytes,
                                      int32_t* status_or, void* stream) {
  if (!spec) return fail(OSTRICH_E_ARG, "loss spec required");
  return rollout_run(ctx, phase, q0, u0, knots, K, basis, T, ckpt_every, loss_body, nullptr, spec, loss_grad, loss,
                     qT, uT, g_q0, g_u0, g_knots, workspace, workspace_bytes, status_or, stream);
}

__global__ void k_adam(double* x, const double* g, double* m, double* v, long n, double lr, double b1, double b2,
                       double eps, double c1, double c2) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double gi = g[i];
  if (!isfinite(gi)) gi = 0.0;  // a diverged rollout leaves the moments to decay
  double mi = b1 * m[i] + (1.0 - b1) * gi;
  double vi = b2 * v[i] + (1.0 - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  x[i] -= lr * (mi / c1) / (::sqrt(vi / c2) + eps);
}

extern "C" int ostrich_spline_controls(const double* basis, const double* knots, int32_t T, int32_t K, int32_t nctrl,
                                       double* ctrl, void* stream) {
  if (!basis || !knots || !ctrl || T < 1 || K < 1 || nctrl < 0) return fail(OSTRICH_E_ARG, "spline controls");
  if (nctrl == 0) return 0;
  hipLaunchKernelGGL(k_ctrl, dim3(nblk((long)T * nctrl, 256)), dim3(256), 0, (hipStream_t)stream, basis, knots, T, K,
                     nctrl, ctrl);
  HIP_OK(hipGetLastError());
  return 0;
}

extern "C" int ostrich_final_loss(const int32_t* body_off, int32_t n_worlds, const double* qT,
                                  const int32_t* loss_body, const double* target, const double* loss_grad,
                                  double* loss, double* gq, void* stream) {
  if (!body_off || !qT || !loss_body || !target || n_worlds < 0) return fail(OSTRICH_E_ARG, "final loss");
  if (n_worlds == 0) return 0;
  hipLaunchKernelGGL(k_loss, dim3(nblk(n_worlds, 256)), dim3(256), 0, (hipStream_t)stream, body_off, n_worlds, qT,
                     loss_body, target, loss_grad, loss, gq, (int32_t*)nullptr);
  HIP_OK(hipGetLastError());
  return 0;
}

extern "C" int ostrich_knot_grad_accumulate(const double* basis, const double* g_ctrl, int32_t k, int32_t K,
                                            int32_t nctrl, double* g_knots, void* stream) {
  if (!basis || !g_ctrl || !g_knots || k < 0 || K < 1 || nctrl < 0) return fail(OSTRICH_E_ARG, "knot gradient");
  if (nctrl == 0) return 0;
  hipLaunchKernelGGL(k_gknots, dim3(nblk((long)nctrl * K, 256)), dim3(256), 0, (hipStream_t)stream, basis, g_ctrl, k,
                     K, nctrl, g_knots);
  HIP_OK(hipGetLastError());
  return 0;
}

namespace {
// Segment copies: the segments of one launch are its grid's y index, each
// copied by a grid-stride loop over its doubles (coalesced 8-byte accesses).
constexpr int kSegsPerLaunch = 32;
struct SegPack {
  const double* src[kSegsPerLaunch];
  double* dst[kSegsPerLaunch];
  int64_t n[kSegsPerLaunch];
};
__global__ void __launch_bounds__(256) k_copy_segments(SegPack p) {
  const int s = blockIdx.y;
  const double* src = p.src[s];
  double* dst = p.dst[s];
  const int64_t n = p.n[s];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}
}  // namespace

extern "C" int ostrich_copy_segments(const ostrich_copy_seg* segs, int32_t n_segs, void* stream) {
  if (n_segs < 0 || (n_segs > 0 && !segs)) return fail(OSTRICH_E_ARG, "copy segments: count or list");
  for (int32_t i = 0; i < n_segs; ++i)
    if (segs[i].n < 0 || (segs[i].n > 0 && (!segs[i].src || !segs[i].dst)))
      return fail(OSTRICH_E_ARG, "copy segment " + std::to_string(i) + ": length or pointer");
  bool launched = false;
  for (int32_t i0 = 0; i0 < n_segs; i0 += kSegsPerLaunch) {
    SegPack p{};
    const int cnt = std::min<int>(kSegsPerLaunch, n_segs - i0);
    int64_t nmax = 0;
    for (int j = 0; j < cnt; ++j) {
      p.src[j] = segs[i0 + j].src;
      p.dst[j] = segs[i0 + j].dst;
      p.n[j] = segs[i0 + j].n;
      nmax = std::max(nmax, segs[i0 + j].n);
    }
    if (nmax == 0) continue;
    const int bx = (int)std::min<int64_t>((nmax + 1023) / 1024, 64);
    hipLaunchKernelGGL(k_copy_segments, dim3(bx, cnt), dim3(256), 0, (hipStream_t)stream, p);
    launched = true;
  }
  if (launched) HIP_OK(hipGetLastError());
  return 0;
}

extern "C" int ostrich_adam(double* x, const double* g, double* m, double* v, int64_t n, double lr, double beta1,
                            double beta2, double eps, int32_t t, void* stream) {
  if (!x || !g || !m || !v || n < 0 || t < 1) return fail(OSTRICH_E_ARG, "adam");
  if (n == 0) return 0;
  double c1 = 1.0 - std::pow(beta1, t), c2 = 1.0 - std::pow(beta2, t);
  hipLaunchKernelGGL(k_adam, dim3(nblk(n, 256)), dim3(256), 0, (hipStream_t)stream, x, g, m, v, (long)n, lr, beta1,
                     beta2, eps, c1, c2);
  HIP_OK(hipGetLastError());
  return 0;
}

extern "C" int ostrich_spline_basis(int32_t T, int32_t K, double h, double* B) {
  if (T < 1 || K < 2 || !B || !(h > 0.0)) return fail(OSTRICH_E_ARG, "spline basis arguments");
  // natural cubic spline: second derivatives m_j from the tridiagonal system
  // dt m_{j-1} + 4 dt m_j + dt m_{j+1} = 6 (y_{j+1} - 2 y_j + y_{j-1}) / dt,
  // m_0 = m_{K-1} = 0, solved by the Thomas algorithm for each unit knot vector
  const double dt = T * h / (K - 1);
  const int n = K - 2;
  std::vector<double> m(K), c(std::max(n, 1)), d(std::max(n, 1));
  for (int j = 0; j < K; ++j) {
    std::fill(m.begin(), m.end(), 0.0);
    if (n > 0) {
      for (int i = 0; i < n; ++i) {
        int k = i + 1;
        double y0 = (k - 1 == j), y1 = (k == j), y2 = (k + 1 == j);
        d[i] = 6.0 * (y2 - 2.0 * y1 + y0) / dt;
      }
      // forward sweep (diagonal 4 dt, off-diagonals dt)
      c[0] = dt / (4.0 * dt);
      d[0] = d[0] / (4.0 * dt);
      for (int i = 1; i < n; ++i) {
        double den = 4.0 * dt - dt * c[i - 1];
        c[i] = dt / den;
        d[i] = (d[i] - dt * d[i - 1]) / den;
      }
      for (int i = n - 1; i >= 0; --i) {
        double v = d[i] - (i + 1 < n ? c[i] * m[i + 2] : 0.0);
        m[i + 1] = v;
      }
    }
    for (int k = 0; k < T; ++k) {
      double t = k * h;
      int i = std::min((int)(t / dt), K - 2);
      double t0 = i * dt, t1 = (i + 1) * dt;
      double a = t1 - t, bq = t - t0;
      double y0 = (i == j), y1 = (i + 1 == j);
      B[k * K + j] = m[i] * a * a * a / (6.0 * dt) + m[i + 1] * bq * bq * bq / (6.0 * dt) +
                     (y0 - m[i] * dt * dt / 6.0) * a / dt + (y1 - m[i + 1] * dt * dt / 6.0) * bq / dt;
    }
  }
  return 0;
}
