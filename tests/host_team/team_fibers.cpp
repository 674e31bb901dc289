// Host build of the library's per-world team procedures with a team of 128
// threads run as fibers: between two barriers the threads run one after
// another in a random order, so a missing barrier shows up as results that
// depend on the schedule.  Each release also checks what the GPU needs and the
// fibers alone would not enforce: a wavefront barrier or cross-lane exchange
// involves the first wavefront only, an exchange (bcast, wmax) has all of its
// lanes present at the same event, a team reduction (sum64, imax) every thread
// of the team, and the threads released from one workgroup barrier have passed
// the same number of barriers (no barrier under a branch that depends on the
// thread).  Violations are counted, not fatal.  Test infrastructure, for CPU
// tests only.
#include <ucontext.h>
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <random>
#include <string>
#include <vector>
#include "newton.hpp"
#include "ostrich.h"
using namespace ost;

// fiber states
enum { RUN = 0, AT_SYNC = 1, DONE = 2, AT_WSYNC = 3, AT_XLANE = 4, AT_REDUCE = 5 };

struct Sched {
  int n;
  std::vector<ucontext_t> ctx;
  ucontext_t main;
  std::vector<std::vector<char>> stacks;
  std::vector<int> state;
  std::vector<long> nbar, nwbar;  // workgroup-level and wavefront-level events passed
  std::vector<double> rv;
  std::vector<int> ri;
  std::mt19937 rng;
  std::function<void(int)> body;
  long phases = 0;
  long violations = 0;
  std::string first;
  void violate(const std::string& what) {
    if (violations++ == 0) first = what;
  }
};
static Sched* gS = nullptr;

struct FiberTeam {
  static constexpr bool kGlobal = false;
  static constexpr bool kRim = true;   // rim-circle contacts compiled in
  Sched* S;
  int r;
  int rank() const { return r; }
  int size() const { return S->n; }
  void wait(int st) const {
    S->state[r] = st;
    if (st == AT_SYNC || st == AT_REDUCE) ++S->nbar[r];
    else ++S->nwbar[r];
    swapcontext(&S->ctx[r], &S->main);
  }
  void sync() const { wait(AT_SYNC); }
  int wsize() const { return 64; }
  void wsync() const { wait(AT_WSYNC); }
  double bcast(double v, int src) const {
    if (src < 0 || src >= 64 || src >= S->n) S->violate("bcast from lane " + std::to_string(src));
    S->rv[r] = v;
    wait(AT_XLANE);
    double o = S->rv[src < 0 ? 0 : (src >= S->n ? S->n - 1 : src)];
    wait(AT_XLANE);
    return o;
  }
  double wmax(double v) const {
    S->rv[r] = v;
    wait(AT_XLANE);
    double m = S->rv[0];
    for (int i = 1; i < 64 && i < S->n; ++i) m = std::max(m, S->rv[i]);
    wait(AT_XLANE);
    return m;
  }
  double sum64(double v, double*) const {
    S->rv[r] = r < 64 ? v : 0.0;
    wait(AT_REDUCE);
    double a[64];
    for (int l = 0; l < 64; ++l) a[l] = l < S->n ? S->rv[l] : 0.0;
    for (int off = 32; off > 0; off >>= 1) {
      double b[64];
      for (int l = 0; l < 64; ++l) b[l] = a[l] + a[l ^ off];
      std::memcpy(a, b, sizeof(a));
    }
    double res = a[0];
    wait(AT_REDUCE);
    return res;
  }
  int imax(int v, double*) const {
    S->ri[r] = v;
    wait(AT_REDUCE);
    int m = S->ri[0];
    for (int i = 1; i < S->n; ++i) m = std::max(m, S->ri[i]);
    wait(AT_REDUCE);
    return m;
  }
};

// Checks one release point: `lanes` are the fibers released together (all at
// one kind of barrier), the others keep waiting.
static void check_release(Sched& S, bool wave_level, int kind) {
  const int n = S.n, w0 = std::min(64, n);
  if (wave_level) {
    long c = -1;
    for (int r = 0; r < n; ++r) {
      const int st = S.state[r];
      if (st != AT_WSYNC && st != AT_XLANE) continue;
      if (r >= 64) S.violate("wavefront barrier reached by thread " + std::to_string(r) + " outside the first wavefront");
      if (st != kind) S.violate("plain wavefront barrier and cross-lane exchange at one release");
      if (c < 0) c = S.nwbar[r];
      else if (S.nwbar[r] != c) S.violate("first-wavefront lanes at different wavefront events");
    }
    if (kind == AT_XLANE)
      for (int r = 0; r < w0; ++r)
        if (S.state[r] != AT_XLANE) S.violate("cross-lane exchange without lane " + std::to_string(r));
    return;
  }
  long c = -1;
  for (int r = 0; r < n; ++r) {
    const int st = S.state[r];
    if (st == DONE) {
      if (kind == AT_REDUCE) S.violate("team reduction after thread " + std::to_string(r) + " finished");
      continue;
    }
    if (st != kind) S.violate("workgroup barrier and team reduction at one release");
    if (c < 0) c = S.nbar[r];
    else if (S.nbar[r] != c) S.violate("threads released from different workgroup barriers");
  }
}

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
  S.state.assign(n, RUN);
  S.nbar.assign(n, 0);
  S.nwbar.assign(n, 0);
  for (int r = 0; r < n; ++r) {
    getcontext(&S.ctx[r]);
    S.ctx[r].uc_stack.ss_sp = S.stacks[r].data();
    S.ctx[r].uc_stack.ss_size = S.stacks[r].size();
    S.ctx[r].uc_link = &S.main;
    makecontext(&S.ctx[r], (void (*)())tramp, 1, r);
  }
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  // all threads start runnable; each phase runs every runnable thread until it
  // waits or finishes, then releases one barrier: a wavefront-level one if any
  // lane waits at one (the other threads keep waiting), else the workgroup's
  while (true) {
    std::shuffle(order.begin(), order.end(), S.rng);
    for (int r : order) {
      if (S.state[r] != RUN) continue;
      swapcontext(&S.main, &S.ctx[r]);
    }
    ++S.phases;
    int wave_kind = 0, group_kind = 0;
    bool alive = false;
    for (int r = 0; r < n; ++r) {
      const int st = S.state[r];
      if (st == AT_WSYNC || st == AT_XLANE) wave_kind = wave_kind ? wave_kind : st;
      if (st == AT_SYNC || st == AT_REDUCE) group_kind = group_kind ? group_kind : st;
      alive |= st != DONE;
    }
    if (!alive) break;
    if (wave_kind) {
      check_release(S, true, wave_kind);
      for (int r = 0; r < n; ++r)
        if (S.state[r] == AT_WSYNC || S.state[r] == AT_XLANE) S.state[r] = RUN;
    } else {
      check_release(S, false, group_kind);
      for (int r = 0; r < n; ++r)
        if (S.state[r] == AT_SYNC || S.state[r] == AT_REDUCE) S.state[r] = RUN;
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
  long violations = 0;
  std::string first;
  // tiered carve (tier_nc > 0): each world first runs with a workspace for tier_nc
  // active contacts and, if the team finds it too small, again with the full one
  int tier_nc = 0;
  Caps caps1;
  std::vector<char> ws1;
  int deferred = 0;
  void take(const Sched& S) {
    if (S.violations && !violations) first = S.first;
    violations += S.violations;
  }
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

// Runs one world's team procedure on a fresh schedule; returns whether it ran to
// the end (a procedure returns false, before writing any output, when the world
// does not fit the carve).  Every thread must return the same.
template <class Body>
static bool run_world(FibCtx* c, unsigned seed, int w, Body body) {
  Sched S;
  S.n = c->team;
  S.rv.assign(c->team, 0.0);
  S.ri.assign(c->team, 0);
  S.rng.seed(seed * 7919 + w);
  std::vector<int> ok(c->team, -1);
  S.body = [&](int r) { ok[r] = body(FiberTeam{&S, r}) ? 1 : 0; };
  run_team(S);
  for (int r = 1; r < c->team; ++r)
    if (ok[r] != ok[0]) S.violate("threads disagree whether the world fits the carve");
  c->take(S);
  return ok[0] == 1;
}

extern "C" void tf_set_tier(void* h, int nc) {
  FibCtx* c = (FibCtx*)h;
  c->tier_nc = nc;
  c->caps1 = c->caps;
  if (nc > 0) {
    c->caps1.nc = nc;
    const int mr = 5 * c->caps.nj + c->caps.nsv + 3 * nc;
    c->caps1.mr = mr < c->caps.mr ? mr : c->caps.mr;
    c->ws1.assign(world_lds_bytes(c->caps1, c->team, SPLIT_LDS, true) + 64, 0);
  }
  c->deferred = 0;
}
extern "C" int tf_deferred(void* h) { return ((FibCtx*)h)->deferred; }

extern "C" void tf_forward(void* h, unsigned seed, const double* q, const double* u, const double* lam,
                           const double* ctrl, double* qn, double* un, double* ln, int* act, int* nact, int* st,
                           int* it, double* rn, double* tape) {
  FibCtx* c = (FibCtx*)h;
  for (int w = 0; w < c->B.n_worlds; ++w) {
    auto fw = [&](std::vector<char>& ws, const Caps& caps) {
      std::memset(ws.data(), 0xFF, ws.size());
      WorldMem M = carve(ws.data(), caps, c->team);
      return run_world(c, seed, w, [&](FiberTeam t) {
        WorldMem Mr = M;
        if (c->P.lin)
          return forward_world<FiberTeam, true>(t, c->B, c->P, caps, w, q, u, lam, ctrl, qn, un, ln, act, nact, st,
                                                it, rn, tape, c->toff.data(), Mr);
        return forward_world(t, c->B, c->P, caps, w, q, u, lam, ctrl, qn, un, ln, act, nact, st, it, rn, tape,
                             c->toff.data(), Mr);
      });
    };
    if (c->tier_nc > 0) {
      if (fw(c->ws1, c->caps1)) continue;
      c->deferred++;
    }
    fw(c->ws, c->caps);
  }
}

extern "C" void tf_adjoint(void* h, unsigned seed, const double* q, const double* u, const double* ctrl,
                           const double* un, const double* ln, const double* tape, const double* gqn,
                           const double* gun, double* gq, double* gu, double* gc, int refine) {
  FibCtx* c = (FibCtx*)h;
  for (int w = 0; w < c->B.n_worlds; ++w) {
    auto bw = [&](std::vector<char>& ws, const Caps& caps) {
      std::memset(ws.data(), 0xFF, ws.size());
      WorldMem M = carve(ws.data(), caps, c->team, SPLIT_LDS, nullptr, true);
      return run_world(c, seed, w, [&](FiberTeam t) {
        WorldMem Mr = M;
        return adjoint_world(t, c->B, c->P, caps, w, q, u, ctrl, un, ln, tape, c->toff.data(), gqn, gun, gq, gu, gc,
                             refine, Mr);
      });
    };
    if (c->tier_nc > 0) {
      if (bw(c->ws1, c->caps1)) continue;
      c->deferred++;
    }
    bw(c->ws, c->caps);
  }
}

// Violations of the GPU's synchronisation rules seen so far (see the top of
// this file); the first one's description goes to buf.
extern "C" long tf_violations(void* h, char* buf, int len) {
  FibCtx* c = (FibCtx*)h;
  if (buf && len > 0) std::snprintf(buf, (size_t)len, "%s", c->first.c_str());
  return c->violations;
}

// The checks above against small team procedures, one correct and three with a
// planted mistake each: 0, correct (first-wavefront exchange beside a waiting
// second wavefront, a barrier, a team reduction); 1, a barrier that only thread
// 0 reaches; 2, an exchange that only lanes 0-9 enter; 3, a team reduction after
// the second wavefront has finished.  Returns the violations counted.
extern "C" long tf_selftest(int kind, int team) {
  Sched S;
  S.n = team;
  S.rv.assign(team, 0.0);
  S.ri.assign(team, 0);
  S.rng.seed(11u + (unsigned)kind);
  S.body = [&](int r) {
    FiberTeam t{&S, r};
    if (kind == 1 && r == 0) t.sync();
    if (kind == 2) {
      if (r < 10) (void)t.bcast(1.0, 3);
    } else if (r < 64) {
      (void)t.bcast((double)r, 3);
    }
    t.sync();
    if (kind == 3 && r >= 64) return;
    (void)t.sum64(1.0, nullptr);
  };
  run_team(S);
  return S.violations;
}
