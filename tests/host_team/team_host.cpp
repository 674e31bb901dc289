// Host build of the library's per-world team procedures with a team of one
// thread, for CPU tests against the oracle.  Test infrastructure: the product
// runs these procedures only on the GPU.  The workspace can be pre-filled
// with garbage so that a read of a never-written entry changes the results.
#include <cmath>
#include <cstring>
#include <vector>
#include "newton.hpp"
#include "ostrich.h"
using namespace ost;

struct SerialTeam {
  static constexpr bool kGlobal = false;
  static constexpr bool kRim = true;   // rim-circle contacts compiled in
  int rank() const { return 0; }
  int size() const { return 1; }
  void sync() const {}
  double sum(double v, double*) const { return v; }
  double sum64(double v, double*) const { return v; }
  int imax(int v, double*) const { return v; }
  int wsize() const { return 1; }
  void wsync() const {}
  double wmax(double v) const { return v; }
  double bcast(double v, int) const { return v; }
};

struct HostCtx {
  Batch B;
  Params P;
  Caps caps;
  int fill;
  std::vector<char> ws;
  std::vector<int64_t> toff;
  // tiered carve (tier_nc > 0): every world is first run with a workspace for
  // tier_nc active contacts and, if it does not fit, again with the full one
  int tier_nc = 0;
  Caps caps1;
  std::vector<char> ws1;
  int deferred = 0;
  std::vector<int32_t> adj;  // per world: the adjoint's status bits of the last th_adjoint
};

extern "C" void* th_create(const ostrich_batch* b, const ostrich_params* p, const int* caps6, const int64_t* toff) {
  HostCtx* c = new HostCtx();
  std::memcpy(&c->B, b, sizeof(Batch));
  c->P.h = p->h;
  for (int k = 0; k < 3; ++k) c->P.g[k] = p->gravity[k];
  c->P.tol = p->tol;
  c->P.eps = p->eps;
  c->P.dg = p->delta_g;
  c->P.dreg = p->delta_reg;
  c->P.dreg_adj = p->delta_reg_adj;
  c->P.d0 = p->delta0;
  c->P.kmax = p->k_max;
  c->P.kmin = p->k_min < p->k_max ? p->k_min : p->k_max;
  c->P.ls_max = p->ls_max;
  c->P.refine = p->refine;
  c->P.truncate = p->truncate;
  c->P.lin = p->linear_solver;
  c->P.lin_iters = p->krylov_iters > 0 ? p->krylov_iters : 16;
  c->caps = Caps{caps6[0], caps6[1], caps6[2], caps6[3], caps6[4], caps6[5]};
  c->fill = 0;
  c->ws.resize(world_lds_bytes(c->caps, 1, SPLIT_LDS, true) + 64);
  c->toff.assign(toff, toff + b->n_worlds + 1);
  return c;
}
extern "C" void th_destroy(void* h) { delete (HostCtx*)h; }
extern "C" void th_set_tier(void* h, int nc) {
  HostCtx* c = (HostCtx*)h;
  c->tier_nc = nc;
  c->caps1 = c->caps;
  if (nc > 0) {
    c->caps1.nc = nc;
    const int mr = 5 * c->caps.nj + c->caps.nsv + 3 * nc;
    c->caps1.mr = mr < c->caps.mr ? mr : c->caps.mr;
    c->ws1.assign(world_lds_bytes(c->caps1, 1, SPLIT_LDS, true) + 64, 0);
  }
  c->deferred = 0;
}
extern "C" int th_deferred(void* h) { return ((HostCtx*)h)->deferred; }
// 0: zeros, 1: all bits set (NaN doubles, -1 integers), 2: 0x7f bytes (huge values)
extern "C" void th_set_fill(void* h, int f) { ((HostCtx*)h)->fill = f; }
static void refill(HostCtx* c) {
  std::memset(c->ws.data(), c->fill == 1 ? 0xFF : (c->fill == 2 ? 0x7F : 0), c->ws.size());
}

extern "C" void th_forward(void* h, const double* q, const double* u, const double* lam, const double* ctrl, double* qn,
                           double* un, double* ln, int* act, int* nact, int* st, int* it, double* rn, double* tape) {
  HostCtx* c = (HostCtx*)h;
  SerialTeam t;
  WorldMem M = carve(c->ws.data(), c->caps, 1);
  for (int w = 0; w < c->B.n_worlds; ++w) {
    refill(c);
    if (c->tier_nc > 0) {
      std::memset(c->ws1.data(), c->fill == 1 ? 0xFF : (c->fill == 2 ? 0x7F : 0), c->ws1.size());
      WorldMem M1 = carve(c->ws1.data(), c->caps1, 1);
      if (forward_world(t, c->B, c->P, c->caps1, w, q, u, lam, ctrl, qn, un, ln, act, nact, st, it, rn, tape,
                        c->toff.data(), M1))
        continue;
      c->deferred++;
    }
    if (c->P.lin)
      forward_world<SerialTeam, true>(t, c->B, c->P, c->caps, w, q, u, lam, ctrl, qn, un, ln, act, nact, st, it, rn,
                                      tape, c->toff.data(), M);
    else
      forward_world(t, c->B, c->P, c->caps, w, q, u, lam, ctrl, qn, un, ln, act, nact, st, it, rn, tape,
                    c->toff.data(), M);
  }
}

extern "C" void th_adjoint(void* h, const double* q, const double* u, const double* ctrl, const double* un,
                           const double* ln, const double* tape, const double* gqn, const double* gun, double* gq,
                           double* gu, double* gc, double* gm, double* gmu, double* gkp, int refine) {
  HostCtx* c = (HostCtx*)h;
  SerialTeam t;
  WorldMem M = carve(c->ws.data(), c->caps, 1, SPLIT_LDS, nullptr, true);
  c->adj.assign(c->B.n_worlds, 0);
  for (int w = 0; w < c->B.n_worlds; ++w) {
    refill(c);
    if (c->tier_nc > 0) {
      std::memset(c->ws1.data(), c->fill == 1 ? 0xFF : (c->fill == 2 ? 0x7F : 0), c->ws1.size());
      WorldMem M1 = carve(c->ws1.data(), c->caps1, 1, SPLIT_LDS, nullptr, true);
      if (adjoint_world(t, c->B, c->P, c->caps1, w, q, u, ctrl, un, ln, tape, c->toff.data(), gqn, gun, gq, gu, gc,
                        refine, M1, gm, gmu, gkp, c->adj.data()))
        continue;
      c->deferred++;
    }
    adjoint_world(t, c->B, c->P, c->caps, w, q, u, ctrl, un, ln, tape, c->toff.data(), gqn, gun, gq, gu, gc, refine, M,
                  gm, gmu, gkp, c->adj.data());
  }
}

// The adjoint's per-world status bits (OSTRICH_ST_ADJ_INEXACT) of the last th_adjoint.
extern "C" void th_adj_status(void* h, int32_t* out) {
  HostCtx* c = (HostCtx*)h;
  for (size_t w = 0; w < c->adj.size(); ++w) out[w] = c->adj[w];
}
