// Host build of the library's per-world team procedures with a team of 128
// threads run as fibers: between two barriers the threads run one after
// another in a random order, so a missing barrier shows up as results that
// depend on the schedule.  Test infrastructure, for CPU tests only.
#include <ucontext.h>
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <random>
#include <vector>
#include "newton.hpp"
#include "ostrich.h"
using namespace ost;

struct Sched {
  int n;
  std::vector<ucontext_t> ctx;
  ucontext_t main;
  std::vector<std::vector<char>> stacks;
  std::vector<int> state;  // 0 runnable, 1 at barrier, 2 done, 3 at wavefront barrier
  std::vector<double> rv;
  std::vector<int> ri;
  std::mt19937 rng;
  std::function<void(int)> body;
  long phases = 0;
};
static Sched* gS = nullptr;

struct FiberTeam {
  static constexpr bool kGlobal = false;
  static constexpr bool kRim = true;   // rim-circle contacts compiled in
  Sched* S;
  int r;
  int rank() const { return r; }
  int size() const { return S->n; }
  void sync() const {
    S->state[r] = 1;
    swapcontext(&S->ctx[r], &S->main);
  }
  int wsize() const { return 64; }
  void wsync() const {
    S->state[r] = 3;
    swapcontext(&S->ctx[r], &S->main);
  }
  double bcast(double v, int src) const {
    S->rv[r] = v;
    wsync();
    double o = S->rv[src];
    wsync();
    return o;
  }
  double wmax(double v) const {
    S->rv[r] = v;
    wsync();
    double m = S->rv[0];
    for (int i = 1; i < 64 && i < S->n; ++i) m = std::max(m, S->rv[i]);
    wsync();
    return m;
  }
  double sum64(double v, double*) const {
    S->rv[r] = r < 64 ? v : 0.0;
    sync();
    double a[64];
    for (int l = 0; l < 64; ++l) a[l] = l < S->n ? S->rv[l] : 0.0;
    for (int off = 32; off > 0; off >>= 1) {
      double b[64];
      for (int l = 0; l < 64; ++l) b[l] = a[l] + a[l ^ off];
      std::memcpy(a, b, sizeof(a));
    }
    double res = a[0];
    sync();
    return res;
  }
  int imax(int v, double*) const {
    S->ri[r] = v;
    sync();
    int m = S->ri[0];
    for (int i = 1; i < S->n; ++i) m = std::max(m, S->ri[i]);
    sync();
    return m;
  }
};

static void tramp(int r) {
  gS->body(r);
  gS->state[r] = 2;
  swapcontext(&gS->ctx[r], &gS->main);
}

static void run_team(Sched& S) {
  gS = &S;
  const int n = S.n;
  S.ctx.assign(n, ucontext_t{});
  S.stacks.assign(n, std::vector<char>(1 << 19));
  S.state.assign(n, 0);
  for (int r = 0; r < n; ++r) {
    getcontext(&S.ctx[r]);
    S.ctx[r].uc_stack.ss_sp = S.stacks[r].data();
    S.ctx[r].uc_stack.ss_size = S.stacks[r].size();
    S.ctx[r].uc_link = &S.main;
    makecontext(&S.ctx[r], (void (*)())tramp, 1, r);
  }
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  // all threads start runnable
  while (true) {
    std::shuffle(order.begin(), order.end(), S.rng);
    for (int r : order) {
      if (S.state[r] != 0) continue;
      swapcontext(&S.main, &S.ctx[r]);
    }
    ++S.phases;
    bool wave = false, alive = false;
    for (int r = 0; r < n; ++r) {
      wave |= S.state[r] == 3;
      alive |= S.state[r] != 2;
    }
    if (!alive) break;
    for (int r = 0; r < n; ++r) {
      if (wave && S.state[r] == 3) S.state[r] = 0;
      if (!wave && S.state[r] == 1) S.state[r] = 0;
    }
  }
}

struct FibCtx {
  Batch B;
  Params P;
  Caps caps;
  int team;
  std::vector<char> ws;
  std::vector<int64_t> toff;
};

extern "C" void* tf_create(const ostrich_batch* b, const ostrich_params* p, const int* caps6, const int64_t* toff,
                           int team) {
  FibCtx* c = new FibCtx();
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
  c->team = team;
  c->ws.resize(world_lds_bytes(c->caps, team, SPLIT_LDS, true) + 64);
  c->toff.assign(toff, toff + b->n_worlds + 1);
  return c;
}
extern "C" void tf_destroy(void* h) { delete (FibCtx*)h; }

extern "C" void tf_forward(void* h, unsigned seed, const double* q, const double* u, const double* lam,
                           const double* ctrl, double* qn, double* un, double* ln, int* act, int* nact, int* st,
                           int* it, double* rn, double* tape) {
  FibCtx* c = (FibCtx*)h;
  for (int w = 0; w < c->B.n_worlds; ++w) {
    Sched S;
    S.n = c->team;
    S.rv.assign(c->team, 0.0);
    S.ri.assign(c->team, 0);
    S.rng.seed(seed * 7919 + w);
    std::memset(c->ws.data(), 0xFF, c->ws.size());
    WorldMem M = carve(c->ws.data(), c->caps, c->team);
    S.body = [&](int r) {
      FiberTeam t{&S, r};
      WorldMem Mr = M;
      if (c->P.lin)
        forward_world<FiberTeam, true>(t, c->B, c->P, c->caps, w, q, u, lam, ctrl, qn, un, ln, act, nact, st, it,
                                       rn, tape, c->toff.data(), Mr);
      else
        forward_world(t, c->B, c->P, c->caps, w, q, u, lam, ctrl, qn, un, ln, act, nact, st, it, rn, tape,
                      c->toff.data(), Mr);
    };
    run_team(S);
  }
}

extern "C" void tf_adjoint(void* h, unsigned seed, const double* q, const double* u, const double* ctrl,
                           const double* un, const double* ln, const double* tape, const double* gqn,
                           const double* gun, double* gq, double* gu, double* gc, int refine) {
  FibCtx* c = (FibCtx*)h;
  for (int w = 0; w < c->B.n_worlds; ++w) {
    Sched S;
    S.n = c->team;
    S.rv.assign(c->team, 0.0);
    S.ri.assign(c->team, 0);
    S.rng.seed(seed * 7919 + w);
    std::memset(c->ws.data(), 0xFF, c->ws.size());
    WorldMem M = carve(c->ws.data(), c->caps, c->team, SPLIT_LDS, nullptr, true);
    S.body = [&](int r) {
      FiberTeam t{&S, r};
      WorldMem Mr = M;
      adjoint_world(t, c->B, c->P, c->caps, w, q, u, ctrl, un, ln, tape, c->toff.data(), gqn, gun, gq, gu, gc, refine,
                    Mr);
    };
    run_team(S);
  }
}
