// HIP kernels and the C ABI of the batched backward-Euler contact step.
//
// One workgroup per world: the world's bodies, rows, Schur matrix and factor
// live in LDS for the whole fused step (contact refresh, Newton loop with
// step length and best-iterate selection, finalisation), so a step is one
// kernel launch for the whole batch.  The adjoint kernel back-solves the
// factor stored by the forward launch.
#include <hip/hip_runtime.h>

#include <algorithm>
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
  __device__ int rank() const { return threadIdx.x; }
  __device__ int size() const { return blockDim.x; }
  __device__ void sync() const { __syncthreads(); }
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
};

__global__ void __launch_bounds__(256) k_forward(ost::Batch B, ost::Params P, ost::Caps caps, const double* q_prev, const double* u_prev,
                          const double* lam_prev, const double* ctrl, double* q_next, double* u_next,
                          double* lam_next, int32_t* act_slot, int32_t* n_act, int32_t* status, int32_t* iters,
                          double* resnorm, double* tape) {
  extern __shared__ __align__(16) char smem[];
  GpuTeam t;
  ost::WorldMem M = ost::carve(smem, caps, blockDim.x);
  for (int w = blockIdx.x; w < B.n_worlds; w += gridDim.x) {
    ost::forward_world(t, B, P, caps, w, q_prev, u_prev, lam_prev, ctrl, q_next, u_next, lam_next, act_slot,
                       n_act, status, iters, resnorm, tape, M);
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) k_adjoint(ost::Batch B, ost::Params P, ost::Caps caps, const double* q_prev, const double* u_prev,
                          const double* ctrl, const double* u_next, const double* lam_next, const double* tape,
                          const double* gq_next, const double* gu_next, double* gq_prev, double* gu_prev,
                          double* g_ctrl, int refine) {
  extern __shared__ __align__(16) char smem[];
  GpuTeam t;
  ost::WorldMem M = ost::carve(smem, caps, blockDim.x);
  for (int w = blockIdx.x; w < B.n_worlds; w += gridDim.x) {
    ost::adjoint_world(t, B, P, caps, w, q_prev, u_prev, ctrl, u_next, lam_next, tape, gq_next, gu_next, gq_prev,
                       gu_prev, g_ctrl, refine, M);
    __syncthreads();
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

// loss |xy(loss_body) - target|^2 and its cotangent on q_T
__global__ void k_loss(const int32_t* body_off, int W, const double* qT, const int32_t* loss_body,
                       const double* target, double* loss, double* gq) {
  int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  int b = body_off[w] + loss_body[w];
  double dx = qT[7 * b] - target[2 * w], dy = qT[7 * b + 1] - target[2 * w + 1];
  if (loss) loss[w] = dx * dx + dy * dy;
  if (gq) {
    gq[7 * b] = 2.0 * dx;
    gq[7 * b + 1] = 2.0 * dy;
  }
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

struct ostrich_ctx {
  ost::Batch B;
  ost::Params P;
  ost::Caps caps;
  int team;
  size_t lds;
  int W, NB, NL, NS, NCTRL;
  int refine;
  std::vector<int32_t> body_off_h;
};

extern "C" const char* ostrich_last_error(void) { return g_err.c_str(); }

static bool is_ptr_ok(const void* p) { return p != nullptr; }

extern "C" int ostrich_ctx_create(const ostrich_batch* b, const ostrich_params* p, ostrich_ctx** out) {
  if (!b || !p || !out) return fail(OSTRICH_E_ARG, "null argument");
  if (b->n_worlds < 1) return fail(OSTRICH_E_ARG, "n_worlds must be >= 1");
  if (!(p->h > 0.0) || p->k_max < 0 || p->k_min < 0 || p->ls_max < 0 || !(p->tol >= 0.0) || !(p->eps > 0.0))
    return fail(OSTRICH_E_ARG, "invalid solver parameters");
  const void* need[] = {b->body_off, b->body_mass, b->body_inertia, b->joint_off, b->ctrl_off, b->slot_off,
                        b->obs_off, b->lam_off, b->contact_cap};
  for (const void* q : need)
    if (!is_ptr_ok(q)) return fail(OSTRICH_E_ARG, "null array in batch");
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
  ost::Caps c{0, 0, 0, 0, 0, 0};
  for (int w = 0; w < W; ++w) {
    int nb = bo[w + 1] - bo[w], nj = jo[w + 1] - jo[w], ns = so[w + 1] - so[w];
    if (nb < 1 || nj < 0 || ns < 0 || cap[w] < 0) return fail(OSTRICH_E_ARG, "malformed offsets");
    int nsv = 0;
    for (int j = jo[w]; j < jo[w + 1]; ++j) nsv += (act[j] == 2 || act[j] == 3);
    c.nb = std::max(c.nb, nb);
    c.nj = std::max(c.nj, nj);
    c.ns = std::max(c.ns, ns);
    c.nc = std::max(c.nc, std::min(cap[w], ns));
    c.nsv = std::max(c.nsv, nsv);
    c.mr = std::max(c.mr, 5 * nj + nsv + 3 * std::min(cap[w], ns));
  }
  c.nc = std::max(c.nc, 1);
  c.mr = std::max(c.mr, 1);
  c.ns = std::max(c.ns, 1);
  int team = p->team > 0 ? p->team : 128;
  if (team != 64 && team != 128 && team != 256) return fail(OSTRICH_E_ARG, "team must be 64, 128 or 256");
  size_t lds = ost::world_lds_bytes(c, team);
  hipDeviceProp_t prop;
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  HIP_OK(hipGetDeviceProperties(&prop, dev));
  if (lds > (size_t)prop.sharedMemPerBlock)
    return fail(OSTRICH_E_UNSUPPORTED, "a world needs " + std::to_string(lds) + " B of LDS, more than " +
                                           std::to_string(prop.sharedMemPerBlock));
  HIP_OK(hipFuncSetAttribute((const void*)k_forward, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  HIP_OK(hipFuncSetAttribute((const void*)k_adjoint, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  ostrich_ctx* ctx = new ostrich_ctx();
  std::memcpy(&ctx->B, b, sizeof(ost::Batch));
  static_assert(sizeof(ost::Batch) == sizeof(ostrich_batch), "batch layouts differ");
  ctx->P.h = p->h;
  for (int k = 0; k < 3; ++k) ctx->P.g[k] = p->gravity[k];
  ctx->P.tol = p->tol;
  ctx->P.eps = p->eps;
  ctx->P.dg = p->delta_g;
  ctx->P.dreg = p->delta_reg;
  ctx->P.d0 = p->delta0;
  ctx->P.kmax = p->k_max;
  ctx->P.kmin = std::min(p->k_min, p->k_max);
  ctx->P.ls_max = p->ls_max;
  ctx->P.refine = p->refine;
  ctx->refine = p->refine;
  ctx->caps = c;
  ctx->team = team;
  ctx->lds = lds;
  ctx->W = W;
  ctx->NB = bo[W];
  ctx->NL = lo[W];
  ctx->NS = so[W];
  ctx->NCTRL = co[W];
  ctx->body_off_h = bo;
  *out = ctx;
  return 0;
}

extern "C" int ostrich_ctx_destroy(ostrich_ctx* ctx) {
  delete ctx;
  return 0;
}

extern "C" int ostrich_ctx_caps(const ostrich_ctx* ctx, int64_t* out) {
  if (!ctx || !out) return fail(OSTRICH_E_ARG, "null argument");
  out[0] = ctx->caps.nb;
  out[1] = ctx->caps.nj;
  out[2] = ctx->caps.ns;
  out[3] = ctx->caps.nc;
  out[4] = ctx->caps.mr;
  out[5] = (int64_t)ctx->lds;
  return 0;
}

extern "C" size_t ostrich_tape_bytes(const ostrich_ctx* ctx) {
  return ctx ? (size_t)ctx->W * ost::tape_doubles(ctx->caps) * sizeof(double) : 0;
}

extern "C" int ostrich_step_forward(ostrich_ctx* ctx, const double* q_prev, const double* u_prev,
                                    const double* lam_prev, const double* ctrl, double* q_next, double* u_next,
                                    double* lam_next, int32_t* act_slot, int32_t* n_act, int32_t* status,
                                    int32_t* iters, double* resnorm, void* tape, void* stream) {
  if (!ctx || !q_prev || !u_prev || !lam_prev || !q_next || !u_next || !lam_next)
    return fail(OSTRICH_E_ARG, "null state pointer");
  if (ctx->NCTRL > 0 && !ctrl) return fail(OSTRICH_E_ARG, "controls required");
  hipLaunchKernelGGL(k_forward, dim3(ctx->W), dim3(ctx->team), ctx->lds, (hipStream_t)stream, ctx->B, ctx->P,
                     ctx->caps, q_prev, u_prev, lam_prev, ctrl, q_next, u_next, lam_next, act_slot, n_act, status,
                     iters, resnorm, (double*)tape);
  HIP_OK(hipGetLastError());
  return 0;
}

extern "C" int ostrich_step_adjoint(ostrich_ctx* ctx, const double* q_prev, const double* u_prev,
                                    const double* ctrl, const double* u_next, const double* lam_next,
                                    const void* tape, const double* gq_next, const double* gu_next, double* gq_prev,
                                    double* gu_prev, double* g_ctrl, int32_t refine, void* stream) {
  if (!ctx || !q_prev || !u_prev || !u_next || !lam_next || !tape || !gq_next || !gu_next || !gq_prev || !gu_prev)
    return fail(OSTRICH_E_ARG, "null pointer");
  if (ctx->NCTRL > 0 && (!ctrl || !g_ctrl)) return fail(OSTRICH_E_ARG, "controls required");
  int rf = refine < 0 ? ctx->refine : refine;
  hipLaunchKernelGGL(k_adjoint, dim3(ctx->W), dim3(ctx->team), ctx->lds, (hipStream_t)stream, ctx->B, ctx->P,
                     ctx->caps, q_prev, u_prev, ctrl, u_next, lam_next, (const double*)tape, gq_next, gu_next,
                     gq_prev, gu_prev, g_ctrl, rf);
  HIP_OK(hipGetLastError());
  return 0;
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
  L.tape = (size_t)c->W * ost::tape_doubles(c->caps);
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

extern "C" int ostrich_rollout(ostrich_ctx* ctx, int32_t phase, const double* q0, const double* u0,
                               const double* knots, int32_t K, const double* basis, int32_t T, int32_t ckpt_every,
                               const int32_t* loss_body, const double* target, double* loss, double* qT,
                               double* uT, double* g_q0, double* g_u0, double* g_knots, void* workspace,
                               size_t workspace_bytes, int32_t* status_or, void* stream_) {
  if (!ctx || !q0 || !u0 || T < 1 || !workspace || !loss_body || !target)
    return fail(OSTRICH_E_ARG, "null argument or T < 1");
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
    hipLaunchKernelGGL(k_loss, dim3(nblk(W, 256)), dim3(256), 0, st, ctx->B.body_off, W, st_q(cur), loss_body,
                       target, loss, (double*)nullptr);
  }
  if (phase & OSTRICH_BACKWARD) {
    if (!g_q0 || !g_u0 || (ctx->NCTRL > 0 && !g_knots)) return fail(OSTRICH_E_ARG, "gradient outputs required");
    double* fin = ckpt_every <= 0 ? ck + (size_t)T * L.S : ck + (size_t)L.n_seg * L.S;
    hipLaunchKernelGGL(k_fill, dim3(nblk(7 * NB, 256)), dim3(256), 0, st, gqa, (long)7 * NB, 0.0);
    hipLaunchKernelGGL(k_fill, dim3(nblk(6 * NB, 256)), dim3(256), 0, st, gua, (long)6 * NB, 0.0);
    if (ctx->NCTRL > 0)
      hipLaunchKernelGGL(k_fill, dim3(nblk((long)ctx->NCTRL * K, 256)), dim3(256), 0, st, g_knots,
                         (long)ctx->NCTRL * K, 0.0);
    hipLaunchKernelGGL(k_loss, dim3(nblk(W, 256)), dim3(256), 0, st, ctx->B.body_off, W, st_q(fin), loss_body,
                       target, (double*)nullptr, gqa);
    double *gq = gqa, *gq2 = gqb, *gu = gua, *gu2 = gub;
    auto adj = [&](double* sm, double* sp, double* tp, int k) -> int {
      int r = ostrich_step_adjoint(ctx, st_q(sm), st_u(sm), ctrl_at(k), st_u(sp), st_l(sp), tp, gq, gu, gq2, gu2,
                                   gc, -1, st);
      if (r) return r;
      if (ctx->NCTRL > 0)
        hipLaunchKernelGGL(k_gknots, dim3(nblk((long)ctx->NCTRL * K, 256)), dim3(256), 0, st, basis, gc, k, K,
                           ctx->NCTRL, g_knots);
      std::swap(gq, gq2);
      std::swap(gu, gu2);
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
