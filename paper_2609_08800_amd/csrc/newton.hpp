// Fused per-world forward step (Newton loop with step length and best-iterate
// selection) and per-world implicit adjoint.
#pragma once

#include "step.hpp"

namespace ost {

// Tape of one world-step: the LU factor of the Schur matrix at the returned
// iterate (band entries of an m x m array with row stride m, inside the
// world's mr_w x mr_w slice), then (regularisation used, m, valid, band).
// World w's tape starts at tape_off[w]; tape_off[w+1] - tape_off[w] = mr_w^2 + 4.
OST_HD size_t tape_doubles_world(int mr_w) { return (size_t)mr_w * mr_w + 4; }

// Visit the band entries (i, j), |i - j| <= bw, of an m x m matrix.
template <class Team, class F> OST_HD void for_band(Team& t, int m, int bw, F f) {
  const int wd = 2 * bw + 1;
  if (wd >= m) {
    for (int e = t.rank(); e < m * m; e += t.size()) {
      const int i = e / m;
      f(i, e - i * m);
    }
  } else {
    for (int e = t.rank(); e < m * wd; e += t.size()) {
      int i = e / wd, j = i - bw + (e - i * wd);
      if (j >= 0 && j < m) f(i, j);
    }
  }
}

// FB argument scales sigma_n = h^2 Abar_nn, sigma_f = h (Abar_t1 + Abar_t2)/2
// from the Delassus diagonal at the warm start u = u-.
template <class Team>
OST_HD void fb_scales(Team& t, const Batch& B, const Params& P, const WorldRef& R, const WorldMem& M,
                      const double* ctrl) {
  evaluate(t, B, P, R, M, ctrl, M.um, M.lam, false);
  const int base = 5 * R.nj + R.nsv;
  for (int c = t.rank(); c < R.nc; c += t.size()) {
    double ad[3];
    for (int k = 0; k < 3; ++k) {
      int i = base + 3 * c + k;
      const double* Jr = M.J + 12 * i;
      double MJ[12], s = 0.0;
      minv6(M, M.r_a[i], Jr, MJ);
      for (int q = 0; q < 6; ++q) s += Jr[q] * MJ[q];
      if (M.r_b[i] >= 0) {
        minv6(M, M.r_b[i], Jr + 6, MJ + 6);
        for (int q = 6; q < 12; ++q) s += Jr[q] * MJ[q];
      }
      ad[k] = s;
    }
    M.c_sn[c] = P.h * P.h * ad[0];
    M.c_sf[c] = P.h * 0.5 * (ad[1] + ad[2]);
  }
  t.sync();
}

// Progress of one world's Newton loop (identical in every thread of the team).
struct FwState {
  double nrm, bn;   // residual norm of the current and of the best iterate
  int have, conv, iters, st, done;
};

// Step set-up of world w: contact refresh, warm start, FB scales and the
// residual at the warm start (Sec. III-A, III-B).  Returns false when the
// world's active contacts do not fit the carve (nothing else is done).
template <class Team>
OST_HD bool fw_begin(Team& t, const Batch& B, const Params& P, WorldRef& R, const double* q_prev,
                     const double* u_prev, const double* lam_prev, const double* ctrl, WorldMem& M, FwState& S) {
  if (!prologue(t, B, P, R, q_prev, u_prev, ctrl, lam_prev, M)) return false;
  clamp_all(t, P, R, M, M.lam);
  fb_scales(t, B, P, R, M, ctrl);
  S.st = M.iscal[1] ? ST_OVERFLOW : 0;
  S.nrm = evaluate(t, B, P, R, M, ctrl, M.u, M.lam, true);
  for (int i = t.rank(); i < 6 * R.nb; i += t.size()) M.ubest[i] = M.u[i];
  for (int i = t.rank(); i < R.m; i += t.size()) M.lambest[i] = M.lam[i];
  S.bn = S.nrm;
  S.have = P.kmin == 0;
  S.conv = 0;
  S.iters = 0;
  S.done = 0;
  if (!isfinite(S.nrm)) {
    S.st |= ST_NONFINITE | ST_BUDGET;
    S.done = 1;
  } else if (S.nrm <= P.tol) {
    S.conv = 1;
    S.done = 1;
  }
  t.sync();
  return true;
}

// Dot product over a fixed partition into 64 lanes (independent of the team size).
template <class Team>
OST_HD double dot64(Team& t, const WorldMem& M, const double* x, const double* y, int n) {
  double s = 0.0;
  for (int l = t.rank(); l < 64; l += t.size())
    for (int i = l; i < n; i += 64) s += x[i] * y[i];
  return t.sum64(s, M.red);
}

// Schur product out = A v without forming A (Eq. (12)): with z = J^T v per
// (body, component), (A v)_i = Y_i . z + sum over row i's group of
// G_lambda,ij v_j / h + dreg Abar_i v_i, Y = G_u M~^-1.
template <class Team>
OST_HD void schur_apply(Team& t, const Params& P, const WorldRef& R, const WorldMem& M, const double* v,
                        double* out) {
  const int nb = R.nb, m = R.m;
  for (int e = t.rank(); e < 6 * nb; e += t.size()) {
    const int b = e / 6, q = e - 6 * b;
    double s = 0.0;
    for (int i = 0; i < m; ++i) {
      if (M.r_a[i] == b) s += M.J[12 * i + q] * v[i];
      if (M.r_b[i] == b) s += M.J[12 * i + 6 + q] * v[i];
    }
    M.kg[e] = s;
  }
  t.sync();
  const double ih = 1.0 / P.h;
  for (int i = t.rank(); i < m; i += t.size()) {
    const double* Y = M.Y + 12 * i;
    const int a = M.r_a[i], b = M.r_b[i], gi = M.r_g[i];
    double s = 0.0;
    for (int k = 0; k < 6; ++k) s += Y[k] * M.kg[6 * a + k];
    if (b >= 0)
      for (int k = 0; k < 6; ++k) s += Y[6 + k] * M.kg[6 * b + k];
    for (int j = gi; j < m && M.r_g[j] == gi; ++j) s += M.Gl[3 * i + (j - gi)] * ih * v[j];
    out[i] = s + P.dreg * M.Abar[i] * v[i];
  }
  t.sync();
}

// Relative residual at which the Newton step's Krylov solve stops.
constexpr double kLinTol = 1e-12;

// Newton direction dlam of Eq. (12) by a matrix-free Krylov solve (the
// paper's iterative alternative to a factor): right-preconditioned restarted
// GMRES, the Jacobi preconditioner diag(A), at most P.lin_iters products
// with A, stop at kLinTol of |rhs|.  A is non-symmetric here (the
// generalized Jacobian), so GMRES takes the place of conjugate residuals.
// The basis and the small least-squares problem live in the Schur matrix's
// storage (`room` doubles), unused in this mode; the restart length is the
// largest that fits.  Returns false on a zero or non-finite diagonal.
template <class Team>
OST_HD bool krylov_direction(Team& t, const Params& P, const WorldRef& R, const WorldMem& M, int room) {
  const int m = R.m;
  int rs = P.lin_iters;
  while (rs > 1 && (size_t)(rs + 1) * (m + rs) + 4 * rs + 2 > (size_t)room) --rs;
  double *V = M.A, *H = V + (size_t)(rs + 1) * m, *cs = H + (size_t)(rs + 1) * rs, *sn = cs + rs;
  double *gv = sn + rs, *y = gv + rs + 1;
  double *dg = M.rmax, *x = M.dlam, *z = M.lamt;
  const double ih = 1.0 / P.h;
  int bad = 0;
  for (int i = t.rank(); i < m; i += t.size()) {  // diag(A)
    const double* Y = M.Y + 12 * i;
    const double* Jr = M.J + 12 * i;
    double s = 0.0;
    for (int k = 0; k < 6; ++k) s += Y[k] * Jr[k];
    if (M.r_b[i] >= 0)
      for (int k = 0; k < 6; ++k) s += Y[6 + k] * Jr[6 + k];
    s += M.Gl[3 * i + (i - M.r_g[i])] * ih + P.dreg * M.Abar[i];
    dg[i] = s;
    x[i] = 0.0;
    V[i] = M.rhs[i];
    bad |= !(isfinite(s) && s != 0.0);
  }
  if (t.imax(bad, M.red)) return false;
  t.sync();
  const double bn = ::sqrt(dot64(t, M, M.rhs, M.rhs, m));
  const double stop = kLinTol * bn;
  double beta = bn;
  int used = 0;
  while (used < P.lin_iters && beta > stop) {
    for (int i = t.rank(); i < m; i += t.size()) V[i] = V[i] / beta;
    if (t.rank() == 0) {
      gv[0] = beta;
      for (int i = 1; i <= rs; ++i) gv[i] = 0.0;
    }
    t.sync();
    int k = 0;
    double res = beta;
    bool more = true;
    while (more && k < rs && used < P.lin_iters && res > stop) {
      const double* vk = V + (size_t)k * m;
      double* w = V + (size_t)(k + 1) * m;
      for (int i = t.rank(); i < m; i += t.size()) z[i] = vk[i] / dg[i];
      t.sync();
      schur_apply(t, P, R, M, z, w);
      ++used;
      for (int i = 0; i <= k; ++i) {  // modified Gram-Schmidt
        const double hik = dot64(t, M, w, V + (size_t)i * m, m);
        for (int e = t.rank(); e < m; e += t.size()) w[e] -= hik * V[(size_t)i * m + e];
        if (t.rank() == 0) H[i * rs + k] = hik;
        t.sync();
      }
      const double hn = ::sqrt(dot64(t, M, w, w, m));
      more = hn > 0.0;
      if (more)
        for (int e = t.rank(); e < m; e += t.size()) w[e] = w[e] / hn;
      if (t.rank() == 0) {
        H[(k + 1) * rs + k] = hn;
        for (int i = 0; i < k; ++i) {
          const double a = H[i * rs + k], b = H[(i + 1) * rs + k];
          H[i * rs + k] = cs[i] * a + sn[i] * b;
          H[(i + 1) * rs + k] = -sn[i] * a + cs[i] * b;
        }
        const double a = H[k * rs + k], b = H[(k + 1) * rs + k];
        const double r = ::sqrt(a * a + b * b);
        cs[k] = r > 0.0 ? a / r : 1.0;
        sn[k] = r > 0.0 ? b / r : 0.0;
        H[k * rs + k] = r;
        H[(k + 1) * rs + k] = 0.0;
        gv[k + 1] = -sn[k] * gv[k];
        gv[k] = cs[k] * gv[k];
      }
      t.sync();
      res = ::fabs(gv[k + 1]);
      ++k;
    }
    if (t.rank() == 0)
      for (int i = k - 1; i >= 0; --i) {
        double s = gv[i];
        for (int j = i + 1; j < k; ++j) s -= H[i * rs + j] * y[j];
        y[i] = H[i * rs + i] != 0.0 ? s / H[i * rs + i] : 0.0;
      }
    t.sync();
    for (int e = t.rank(); e < m; e += t.size()) {  // x += D^-1 V y
      double s = 0.0;
      for (int i = 0; i < k; ++i) s += y[i] * V[(size_t)i * m + e];
      x[e] += s / dg[e];
    }
    t.sync();
    if (!more || !(res > stop) || used >= P.lin_iters) break;
    schur_apply(t, P, R, M, x, V);  // restart from the true residual rhs - A x
    ++used;
    for (int e = t.rank(); e < m; e += t.size()) V[e] = M.rhs[e] - V[e];
    t.sync();
    beta = ::sqrt(dot64(t, M, V, V, m));
  }
  return true;
}

// Newton iteration k (Eqs. (12)-(13)): factor, solve, step length, friction
// clamp, best-iterate bookkeeping (Sec. III-C).  Nothing happens once done.
template <class Team, bool kKrylov = false>
OST_HD void fw_iteration(Team& t, const Batch& B, const Params& P, const WorldRef& R, const double* ctrl,
                         WorldMem& M, FwState& S, int k, int room = 0) {
  if (S.done) return;
  const int nb = R.nb, m = R.m;
  if (kKrylov) {  // matrix-free direction; the Schur matrix is never formed
    schur_rhs(t, P, R, M);
    if (!krylov_direction(t, P, R, M, room)) {
      S.st |= ST_NONFINITE;
      S.done = 1;
      return;
    }
  } else {
    double dreg;
    if (!factor(t, P, R, M, true, P.dreg, &dreg, &S.st)) {
      S.st |= ST_NONFINITE;
      S.done = 1;
      return;
    }
    for (int i = t.rank(); i < m; i += t.size()) M.dlam[i] = M.rhs[i];
    t.sync();
    lu_solve(t, R, M, M.dlam, false);
  }
  // Eq. (13): du = M~^-1 (h J^T dlambda - r_dyn), force per (body, component)
  for (int e = t.rank(); e < 6 * nb; e += t.size()) {
    int b = e / 6, q = e - 6 * b;
    double v = -M.rdyn[e];
    for (int i0 = 0; i0 < m; i0 += 4) {  // rows in fours: the loads first, then the sum in row order
      int ra[4], rb[4];
      double ja[4], jb[4], dl[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + r < m ? i0 + r : m - 1;
        ra[r] = i0 + r < m ? M.r_a[i] : -2;
        rb[r] = i0 + r < m ? M.r_b[i] : -2;
        ja[r] = M.J[12 * i + q];
        jb[r] = M.J[12 * i + 6 + q];
        dl[r] = M.dlam[i];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (ra[r] == b) v += P.h * ja[r] * dl[r];
        if (rb[r] == b) v += P.h * jb[r] * dl[r];
      }
    }
    M.kg[e] = v;
  }
  t.sync();
  for (int b = t.rank(); b < nb; b += t.size()) minv6(M, b, M.kg + 6 * b, M.du + 6 * b);
  t.sync();
  // step length: halve until the residual decreases by (1 - 1e-4 alpha), else the best trial
  // (the full step is evaluated with the Newton rows, which are reused when it is accepted)
  double alpha = 1.0, best_a = 1.0, best_n = INFINITY;
  bool first_ok = false;
  for (int ls = 0; ls <= P.ls_max; ++ls) {
    for (int i = t.rank(); i < 6 * nb; i += t.size()) M.ut[i] = M.u[i] + alpha * M.du[i];
    for (int i = t.rank(); i < m; i += t.size()) M.lamt[i] = M.lam[i] + alpha * M.dlam[i];
    t.sync();
    clamp_all(t, P, R, M, M.lamt);
    double tn = evaluate(t, B, P, R, M, ctrl, M.ut, M.lamt, ls == 0);
    bool ok = tn <= (1.0 - 1e-4 * alpha) * S.nrm;
    if (tn < best_n || ok) { best_n = tn; best_a = alpha; }
    if (ok) { first_ok = ls == 0; break; }
    alpha *= 0.5;
  }
  if (first_ok) {
    for (int i = t.rank(); i < 6 * nb; i += t.size()) M.u[i] = M.ut[i];
    for (int i = t.rank(); i < m; i += t.size()) M.lam[i] = M.lamt[i];
    t.sync();
    S.nrm = best_n;
  } else {
    for (int i = t.rank(); i < 6 * nb; i += t.size()) M.u[i] = M.u[i] + best_a * M.du[i];
    for (int i = t.rank(); i < m; i += t.size()) M.lam[i] = M.lam[i] + best_a * M.dlam[i];
    t.sync();
    clamp_all(t, P, R, M, M.lam);
    S.nrm = evaluate(t, B, P, R, M, ctrl, M.u, M.lam, true);
  }
  S.iters = k;
  if (!isfinite(S.nrm)) {
    S.st |= ST_NONFINITE;
    S.done = 1;
    return;
  }
  bool take = S.nrm <= P.tol || (k >= P.kmin && (!S.have || S.nrm < S.bn));
  if (take) {
    for (int i = t.rank(); i < 6 * nb; i += t.size()) M.ubest[i] = M.u[i];
    for (int i = t.rank(); i < m; i += t.size()) M.lambest[i] = M.lam[i];
    S.bn = S.nrm;
    S.have = 1;
    t.sync();
  }
  if (S.nrm <= P.tol) {
    S.conv = 1;
    S.done = 1;
  }
}

// Finalisation of world w (Sec. III-C, III-D): the Schur factor at the
// returned iterate to the tape, q+ by Eq. (1) with the quaternion
// renormalised, lambda+ in slot order, status.
template <class Team>
OST_HD void fw_end(Team& t, const Batch& B, const Params& P, const WorldRef& R, int w, const double* ctrl,
                   double* q_next, double* u_next, double* lam_next, int32_t* act_slot, int32_t* n_act,
                   int32_t* status, int32_t* iters_out, double* resnorm, double* tape, const int64_t* tape_off,
                   WorldMem& M, const FwState& S0, int32_t* hist = nullptr) {
  const int nb = R.nb, m = R.m;
  int st = S0.st;
  const int iters = S0.iters;
  const double bn = S0.bn;
  const bool conv = S0.conv;
  st |= conv ? ST_CONVERGED : ST_BUDGET;
  // the tape holds the factor of the Schur matrix at the returned iterate
  if (tape) {
    for (int i = t.rank(); i < 6 * nb; i += t.size()) M.u[i] = M.ubest[i];
    for (int i = t.rank(); i < m; i += t.size()) M.lam[i] = M.lambest[i];
    t.sync();
    evaluate(t, B, P, R, M, ctrl, M.u, M.lam, true);
    // the adjoint's factor, regularised by its own dreg_adj: the root does not
    // depend on the Newton iterations' regularisation, the adjoint would
    double dreg = P.dreg_adj;
    int fst = 0;
    bool ok = factor(t, P, R, M, false, P.dreg_adj, &dreg, &fst);
    double* tw = tape + tape_off[w];
    const int ld = lda(m);  // the tape keeps row stride m
    for_band(t, m, R.bw, [&](int i, int j) { tw[i * m + j] = M.A[i * ld + j]; });
    if (t.rank() == 0) {
      double* tr = tape + tape_off[w + 1] - 4;
      tr[0] = dreg;
      tr[1] = m;
      tr[2] = ok ? 1.0 : 0.0;
      tr[3] = R.bw;
    }
  }
  // q+ = q- + h G(q-) u* with the quaternion renormalised (Eq. (1))
  for (int b = t.rank(); b < nb; b += t.size()) {
    const double* q = M.qm + 7 * b;
    const double* u = M.ubest + 6 * b;
    double* qo = q_next + 7 * (R.b0 + b);
    for (int k = 0; k < 3; ++k) qo[k] = q[k] + P.h * u[k];
    v3<double> wv{u[3], u[4], u[5]}, qv{q[3], q[4], q[5]};
    v3<double> dv = wv * q[6] + cross(wv, qv);
    double dw = -dot(wv, qv);
    double r4[4] = {q[3] + 0.5 * P.h * dv.x, q[4] + 0.5 * P.h * dv.y, q[5] + 0.5 * P.h * dv.z, q[6] + 0.5 * P.h * dw};
    double n = ::sqrt(r4[0] * r4[0] + r4[1] * r4[1] + r4[2] * r4[2] + r4[3] * r4[3]);
    for (int k = 0; k < 4; ++k) qo[3 + k] = r4[k] / n;
    for (int k = 0; k < 6; ++k) u_next[6 * (R.b0 + b) + k] = u[k];
  }
  // every output entry is written exactly once: multipliers of inactive slots
  // are zero, active slots take their row of the returned iterate
  const int lam_len = B.lam_off[w + 1] - R.l0;
  const int base = 5 * R.nj + R.nsv;
  for (int i = t.rank(); i < lam_len; i += t.size()) {
    double v = 0.0;
    if (i < base) {
      v = M.lambest[i];
    } else {
      int s = (i - base) / 3, c = M.s_act[s];
      if (c >= 0) v = M.lambest[base + 3 * c + (i - base) % 3];
    }
    lam_next[R.l0 + i] = v;
  }
  if (act_slot)
    for (int c = t.rank(); c < R.ns; c += t.size()) act_slot[R.s0 + c] = c < R.nc ? M.c_slot[c] : -1;
  if (t.rank() == 0) {
    if (n_act) n_act[w] = R.nc;
    if (status) status[w] = st;
    if (iters_out) iters_out[w] = iters;
    if (resnorm) resnorm[w] = bn;
    if (hist) {  // for the launch plan of the next step: active contacts and Newton iterations
      hist[2 * w] = R.nc;
      hist[2 * w + 1] = iters;
    }
  }
  t.sync();
}

// One backward-Euler step of world w (Sec. III-A..C), fused: set-up, the
// Newton loop and finalisation in one pass of the team.  Returns false, with
// no output written, when the world's active contacts exceed the carve.
template <class Team, bool kKrylov = false>
OST_HD bool forward_world(Team& t, const Batch& B, const Params& P, const Caps& caps, int w, const double* q_prev,
                          const double* u_prev, const double* lam_prev, const double* ctrl, double* q_next,
                          double* u_next, double* lam_next, int32_t* act_slot, int32_t* n_act, int32_t* status,
                          int32_t* iters_out, double* resnorm, double* tape, const int64_t* tape_off,
                          WorldMem& M, int32_t* hist = nullptr) {
  WorldRef R = world_ref(B, w);
  FwState S;
  if (!fw_begin(t, B, P, R, q_prev, u_prev, lam_prev, ctrl, M, S)) return false;
  const int room = (int)M.a_room;  // doubles of the Schur matrix's storage
  for (int k = 1; k <= P.kmax && !S.done; ++k) fw_iteration<Team, kKrylov>(t, B, P, R, ctrl, M, S, k, room);
  fw_end(t, B, P, R, w, ctrl, q_next, u_next, lam_next, act_slot, n_act, status, iters_out, resnorm, tape, tape_off,
         M, S, hist);
  return true;
}

// Loop state kept in the world's workspace between the launches of the plain
// path (one launch per world per Newton iteration).
OST_HD void fw_store(const WorldMem& M, const FwState& S) {
  M.dscal[0] = S.nrm;
  M.dscal[1] = S.bn;
  M.iscal[4] = S.have;
  M.iscal[5] = S.conv;
  M.iscal[6] = S.iters;
  M.iscal[7] = S.st;
  M.iscal[8] = S.done;
}
OST_HD FwState fw_load(const WorldMem& M) {
  FwState S;
  S.nrm = M.dscal[0];
  S.bn = M.dscal[1];
  S.have = M.iscal[4];
  S.conv = M.iscal[5];
  S.iters = M.iscal[6];
  S.st = M.iscal[7];
  S.done = M.iscal[8];
  return S;
}
// The world view after its prologue, rebuilt from the workspace.
OST_HD WorldRef world_ref_after(const Batch& B, const WorldMem& M, int w) {
  WorldRef R = world_ref(B, w);
  R.nc = M.iscal[0];
  R.m = 5 * R.nj + R.nsv + 3 * R.nc;
  R.bw = M.iscal[3];
  return R;
}

// --------------------------------------------------------------------------
// Adjoint.
// --------------------------------------------------------------------------

// Solve the transposed Newton system [[M~, G_u^T], [-h J, G_lambda^T]] [w_u; w_l]
// = [-b; 0] with the stored factor: A^T w_l = -J M~^-1 b,
// w_u = -(M~^-1 b + (G_u M~^-1)^T w_l)   (Eqs. (18)-(19)).
template <class Team>
OST_HD void adjoint_solve(Team& t, const WorldRef& R, const WorldMem& M, const double* b, double* wu, double* wl) {
  const int nb = R.nb, m = R.m;
  for (int q = t.rank(); q < nb; q += t.size()) minv6(M, q, b + 6 * q, M.kg + 6 * q);  // M~^-1 b
  t.sync();
  for (int i = t.rank(); i < m; i += t.size()) {
    const double* Jr = M.J + 12 * i;
    int a = M.r_a[i], c = M.r_b[i];
    double s = 0.0;
    for (int k = 0; k < 6; ++k) s += Jr[k] * M.kg[6 * a + k];
    if (c >= 0) for (int k = 0; k < 6; ++k) s += Jr[6 + k] * M.kg[6 * c + k];
    wl[i] = -s;
  }
  t.sync();
  lu_solve(t, R, M, wl, true);
  for (int e = t.rank(); e < 6 * nb; e += t.size()) {
    int q = e / 6, k = e - 6 * q;
    double s = M.kg[e];
    for (int i0 = 0; i0 < m; i0 += 4) {  // rows in fours: the loads first, then the sum in row order
      int ra[4], rb[4];
      double ya[4], yb[4], w[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + r < m ? i0 + r : m - 1;
        ra[r] = i0 + r < m ? M.r_a[i] : -2;
        rb[r] = i0 + r < m ? M.r_b[i] : -2;
        ya[r] = M.Y[12 * i + k];
        yb[r] = M.Y[12 * i + 6 + k];
        w[r] = wl[i];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (ra[r] == q) s += ya[r] * w[r];
        if (rb[r] == q) s += yb[r] * w[r];
      }
    }
    wu[e] = -s;
  }
  t.sync();
}

// Product with the transposed geometric stiffness, out = K^T v, where K =
// d(J(u)^T lambda)/du at the converged step: the stored factor leaves K out of
// the Jacobian.  Each thread seeds one velocity component with a dual number.
template <class Team>
OST_HD void stiffness_t(Team& t, const Batch& B, const Params& P, const WorldRef& R, WorldMem& M,
                        const double* ctrl, const double* v, double* out) {
  for (int p = t.rank(); p < 6 * R.nb; p += t.size()) {
    int beta = p / 6, comp = p % 6;
    double s = 0.0;
    const int ng = n_groups(R);
    for (int g = 0; g < ng; ++g) {
      int row = group_row(R, g);
      int a = M.r_a[row], c = M.r_b[row];
      if (a != beta && c != beta) continue;
      int kind = M.r_kind[row];
      int n = kind == RK_CONTACT ? 3 : 1;
      double target = kind == RK_SERVO ? M.sv_in[row - 5 * R.nj] : 0.0;
      GroupIn<double> in = group_in_lds(M, row, M.u, M.lam, target);
      dual ua[6], ub[6], lg[3];
      for (int k = 0; k < 6; ++k) {
        ua[k] = dual(M.u[6 * a + k], (a == beta && k == comp) ? 1.0 : 0.0);
        ub[k] = c >= 0 ? dual(M.u[6 * c + k], (c == beta && k == comp) ? 1.0 : 0.0) : dual(0.0);
      }
      #pragma unroll
      for (int k = 0; k < 3; ++k) if (k < n) lg[k] = dual(M.lam[row + k]);
      GroupIn<dual> ind;
      ind.xa = v3<dual>{in.xa.x, in.xa.y, in.xa.z};
      ind.xb = v3<dual>{in.xb.x, in.xb.y, in.xb.z};
      for (int k = 0; k < 9; ++k) { ind.Ra.a[k] = in.Ra.a[k]; ind.Rb.a[k] = in.Rb.a[k]; }
      ind.ua = ua;
      ind.ub = c >= 0 ? ub : nullptr;
      ind.lg = lg;
      ind.target = dual(target);
      ind.fr = lift_frame(in.fr);
      dual rd[3], Jd[36];
      double Dd[3];
      eval_row_group<dual, Team::kRim>(B, P, R, M, row, ind, rd, Jd, Dd);
      #pragma unroll
      for (int k = 0; k < 3; ++k) if (k < n) {
        double jw = 0.0;
        for (int q = 0; q < 6; ++q) jw += Jd[12 * k + q].d * v[6 * a + q];
        if (c >= 0) for (int q = 0; q < 6; ++q) jw += Jd[12 * k + 6 + q].d * v[6 * c + q];
        s += M.lam[row + k] * jw;
      }
    }
    out[p] = s;
  }
  t.sync();
}

// out = v + S(h K^T v): the velocity block of the exact adjoint system after
// the stored factor's solve S (the velocity part of adjoint_solve) is applied.
template <class Team>
OST_HD void kry_apply(Team& t, const Batch& B, const Params& P, const WorldRef& R, WorldMem& M,
                      const double* ctrl, const double* v, double* out) {
  const int n = 6 * R.nb;
  stiffness_t(t, B, P, R, M, ctrl, v, M.ubest);
  for (int p = t.rank(); p < n; p += t.size()) M.ubest[p] = P.h * M.ubest[p];
  t.sync();
  adjoint_solve(t, R, M, M.ubest, out, M.lamt);
  for (int p = t.rank(); p < n; p += t.size()) out[p] += v[p];
  t.sync();
}

// Relative residual at which the adjoint's Krylov solve stops.
constexpr double kKryTol = 1e-12;

// Velocity part x of the exact adjoint, (I + S h K^T) x = c with c = S b the
// stored factor's solution: restarted GMRES (restart kKry, modified
// Gram-Schmidt, Givens rotations) from x = 0, at most `max_apply` operator
// applications, stopping at a residual of kKryTol |c|.  The residual never
// grows, whatever the spectral radius of S h K^T (a fixed-point iteration
// on the same operator diverges once that radius reaches one).  Returns
// whether the stop was reached (or the Krylov space holds the solution);
// false when the applications ran out first or a value was not finite.
template <class Team>
OST_HD bool adjoint_krylov(Team& t, const Batch& B, const Params& P, const WorldRef& R, WorldMem& M,
                          const double* ctrl, const double* c, int max_apply) {
  const int n = 6 * R.nb;
  double *V = M.kv, *x = M.kx, *H = M.kh, *cs = M.kcs, *sn = M.ksn, *gv = M.kgv, *y = M.ky;
  const double cn = ::sqrt(dot64(t, M, c, c, n));
  const double stop = kKryTol * cn;
  for (int e = t.rank(); e < n; e += t.size()) { x[e] = 0.0; V[e] = c[e]; }
  t.sync();
  double beta = cn;  // |c - A x| at x = 0
  int used = 0;
  bool ok = cn <= stop;
  while (used < max_apply && beta > stop) {
    for (int e = t.rank(); e < n; e += t.size()) V[e] = V[e] / beta;
    if (t.rank() == 0) {
      gv[0] = beta;
      for (int i = 1; i <= kKry; ++i) gv[i] = 0.0;
    }
    t.sync();
    int k = 0;
    double res = beta;
    bool more = true;
    while (more && k < kKry && used < max_apply && res > stop) {
      double* w = V + (size_t)(k + 1) * n;
      kry_apply(t, B, P, R, M, ctrl, V + (size_t)k * n, w);
      ++used;
      for (int i = 0; i <= k; ++i) {
        const double hik = dot64(t, M, w, V + (size_t)i * n, n);
        for (int e = t.rank(); e < n; e += t.size()) w[e] -= hik * V[(size_t)i * n + e];
        if (t.rank() == 0) H[i * kKry + k] = hik;
        t.sync();
      }
      const double hn = ::sqrt(dot64(t, M, w, w, n));
      more = hn > 0.0;  // zero: the Krylov space holds the solution; not finite: give up
      if (more)
        for (int e = t.rank(); e < n; e += t.size()) w[e] = w[e] / hn;
      if (t.rank() == 0) {
        H[(k + 1) * kKry + k] = hn;
        for (int i = 0; i < k; ++i) {
          const double a = H[i * kKry + k], b = H[(i + 1) * kKry + k];
          H[i * kKry + k] = cs[i] * a + sn[i] * b;
          H[(i + 1) * kKry + k] = -sn[i] * a + cs[i] * b;
        }
        const double a = H[k * kKry + k], b = H[(k + 1) * kKry + k];
        const double r = ::sqrt(a * a + b * b);
        cs[k] = r > 0.0 ? a / r : 1.0;
        sn[k] = r > 0.0 ? b / r : 0.0;
        H[k * kKry + k] = r;
        H[(k + 1) * kKry + k] = 0.0;
        gv[k + 1] = -sn[k] * gv[k];
        gv[k] = cs[k] * gv[k];
      }
      t.sync();
      res = ::fabs(gv[k + 1]);
      ok = res <= stop || hn == 0.0;
      ++k;
    }
    if (t.rank() == 0)  // the k x k triangle: H y = g
      for (int i = k - 1; i >= 0; --i) {
        double s = gv[i];
        for (int j = i + 1; j < k; ++j) s -= H[i * kKry + j] * y[j];
        y[i] = H[i * kKry + i] != 0.0 ? s / H[i * kKry + i] : 0.0;
      }
    t.sync();
    for (int e = t.rank(); e < n; e += t.size()) {
      double s = x[e];
      for (int i = 0; i < k; ++i) s += y[i] * V[(size_t)i * n + e];
      x[e] = s;
    }
    t.sync();
    if (!more || !(res > stop) || used >= max_apply) break;
    kry_apply(t, B, P, R, M, ctrl, x, V);  // restart from the true residual c - A x
    ++used;
    for (int e = t.rank(); e < n; e += t.size()) V[e] = c[e] - V[e];
    t.sync();
    beta = ::sqrt(dot64(t, M, V, V, n));
    ok = beta <= stop;
  }
  return ok;
}

// Dual input of a group with body data recomputed from q- (seeded), used by
// the pose pull-back.  seed_body / seed_comp select the seeded q- component.
OST_HD void dual_pose(const double* q, int seeded, int comp, v3<dual>& x, m3<dual>& Rm) {
  dual c[7];
  for (int k = 0; k < 7; ++k) c[k] = dual(q[k], seeded && comp == k ? 1.0 : 0.0);
  x = v3<dual>{c[0], c[1], c[2]};
  Rm = quat_to_R(c[3], c[4], c[5], c[6]);
}

// Implicit adjoint of one world-step (Sec. III-D): loss cotangents on s+ to
// cotangents on q-, u- and the controls, through the exact implicit-function
// Jacobian, solved by the Krylov method on the stored factor with at most
// `refine` operator applications (ST_ADJ_INEXACT is ORed into adj_status[w]
// when it ends above its stop).  Returns false, with no output written, when
// the world's active contacts exceed the carve.
template <class Team>
OST_HD bool adjoint_world(Team& t, const Batch& B, const Params& P, const Caps& caps, int w, const double* q_prev,
                          const double* u_prev, const double* ctrl, const double* u_next, const double* lam_next,
                          const double* tape, const int64_t* tape_off, const double* gq_next,
                          const double* gu_next, double* gq_prev, double* gu_prev, double* g_ctrl, int refine,
                          WorldMem& M, double* g_mass = nullptr, double* g_mu = nullptr, double* g_kp = nullptr,
                          int32_t* adj_status = nullptr) {
  WorldRef R = world_ref(B, w);
  const double h = P.h;
  if (!prologue(t, B, P, R, q_prev, u_prev, ctrl, lam_next, M)) return false;
  fb_scales(t, B, P, R, M, ctrl);
  const int nb = R.nb, m = R.m;
  for (int i = t.rank(); i < 6 * nb; i += t.size()) M.u[i] = u_next[6 * R.b0 + i];
  t.sync();
  evaluate(t, B, P, R, M, ctrl, M.u, M.lam, true);
  const double* tw = tape + tape_off[w];
  const double* tr = tape + tape_off[w + 1] - 4;
  if (tr[2] == 1.0 && (int)tr[1] == m && (int)tr[3] == R.bw) {
    const int ld = lda(m);
    for_band(t, m, R.bw, [&](int i, int j) { M.A[i * ld + j] = tw[i * m + j]; });
    t.sync();
  } else {  // no usable stored factor: factor here
    double dreg;
    int fst = 0;
    factor(t, P, R, M, false, P.dreg_adj, &dreg, &fst);
  }
  // loss cotangent on the raw q+ (through the renormalisation) and the total
  // velocity cotangent b = g_u + h G(q-)^T g_q
  for (int b = t.rank(); b < nb; b += t.size()) {
    const double* q = M.qm + 7 * b;
    const double* u = M.u + 6 * b;
    const double* g = gq_next + 7 * (R.b0 + b);
    v3<double> wv{u[3], u[4], u[5]}, qv{q[3], q[4], q[5]};
    v3<double> dv = wv * q[6] + cross(wv, qv);
    double dw = -dot(wv, qv);
    double r4[4] = {q[3] + 0.5 * h * dv.x, q[4] + 0.5 * h * dv.y, q[5] + 0.5 * h * dv.z, q[6] + 0.5 * h * dw};
    double n = ::sqrt(r4[0] * r4[0] + r4[1] * r4[1] + r4[2] * r4[2] + r4[3] * r4[3]);
    double qh[4] = {r4[0] / n, r4[1] / n, r4[2] / n, r4[3] / n};
    double dq = qh[0] * g[3] + qh[1] * g[4] + qh[2] * g[5] + qh[3] * g[6];
    double* gr = M.gq + 7 * b;
    for (int k = 0; k < 3; ++k) gr[k] = g[k];
    for (int k = 0; k < 4; ++k) gr[3 + k] = (g[3 + k] - qh[k] * dq) / n;
    const double* gu = gu_next + 6 * (R.b0 + b);
    double* bb = M.du + 6 * b;  // b
    for (int k = 0; k < 3; ++k) bb[k] = gu[k] + h * gr[k];
    v3<double> gv{gr[3], gr[4], gr[5]};
    v3<double> t3 = gv * q[6] + cross(qv, gv) - qv * gr[6];
    bb[3] = gu[3] + 0.5 * h * t3.x;
    bb[4] = gu[4] + 0.5 * h * t3.y;
    bb[5] = gu[5] + 0.5 * h * t3.z;
    for (int k = 0; k < 6; ++k) M.rdyn[6 * b + k] = bb[k];  // keep b
  }
  t.sync();
  double* wu = M.ut;
  double* wl = M.dlam;
  adjoint_solve(t, R, M, M.du, wu, wl);
  // refinement towards the exact Jacobian, whose velocity block adds the
  // geometric stiffness h K that the factor leaves out: the Krylov solve gives
  // the velocity part x, then one solve with [b - h K^T x; 0] gives w_u, w_l
  if (refine > 0 && M.kv) {
    const bool solved = adjoint_krylov(t, B, P, R, M, ctrl, wu, refine);
    if (!solved && adj_status && t.rank() == 0) adj_status[w] |= ST_ADJ_INEXACT;
    stiffness_t(t, B, P, R, M, ctrl, M.kx, M.kg);
    for (int p = t.rank(); p < 6 * nb; p += t.size()) M.ubest[p] = M.rdyn[p] - h * M.kg[p];
    t.sync();
    adjoint_solve(t, R, M, M.ubest, wu, wl);
  }
  // pull-back, Eq. (17): dL/dxi = w^T D dF/dxi, plus the direct kinematic term
  for (int b = t.rank(); b < nb; b += t.size()) {  // u-: -M~ w_u - h (df_gyro/dw-)^T w_u
    const double* um = M.um + 6 * b;
    const double* wb = wu + 6 * b;
    const double* Iw = M.Iw + 9 * b;
    double* go = gu_prev + 6 * (R.b0 + b);
    for (int k = 0; k < 3; ++k) go[k] = -M.mass[b] * wb[k];
    v3<double> wm{um[3], um[4], um[5]}, ww{wb[3], wb[4], wb[5]};
    auto Iv = [&](const v3<double>& v) {
      return v3<double>{Iw[0] * v.x + Iw[1] * v.y + Iw[2] * v.z, Iw[3] * v.x + Iw[4] * v.y + Iw[5] * v.z,
                        Iw[6] * v.x + Iw[7] * v.y + Iw[8] * v.z};
    };
    v3<double> mw = Iv(ww);
    v3<double> gT = cross(ww, Iv(wm)) + Iv(cross(wm, ww));  // (df/dw)^T w, f = -w x (I w)
    go[3] = -mw.x - h * gT.x;
    go[4] = -mw.y - h * gT.y;
    go[5] = -mw.z - h * gT.z;
  }
  if (t.rank() == 0 && g_ctrl) {  // controls: torque and servo target
    int c = 0, sv = 0;
    for (int j = 0; j < R.nj; ++j) {
      int act = B.joint_act[R.j0 + j];
      int a = B.joint_body[2 * (R.j0 + j)], b = B.joint_body[2 * (R.j0 + j) + 1];
      double g = 0.0;
      if (act == 1 || act == 3) {
        v3<double> ax = mul(ldm(M.Rm + 9 * a), ldv(B.joint_frame + 18 * (R.j0 + j) + 15));
        for (int k = 0; k < 3; ++k) g += -h * at(ax, k) * (wu[6 * b + 3 + k] - wu[6 * a + 3 + k]);
      }
      if (act == 2) g = -wl[5 * R.nj + sv];
      if (act == 4) {  // the servo row holds -alpha k_p theta*
        const double kp = B.joint_kp[R.j0 + j];
        g = -(kp / (B.joint_kd[R.j0 + j] + h * kp)) * wl[5 * R.nj + sv];
      }
      if (act == 2 || act == 3 || act == 4) ++sv;
      if (act) g_ctrl[R.c0 + c++] = g;
    }
  }
  // q-: forward duals over the 7 components of every body's pose; with
  // P.truncate the contact groups, whose geometry is then held fixed within
  // the step, contribute nothing
  for (int p = t.rank(); p < 7 * nb; p += t.size()) {
    int beta = p / 7, comp = p % 7;
    double s = 0.0;
    // body terms of every body (inertia at q-, gyroscopic term, actuator axes)
    for (int b = 0; b < nb; ++b) {
      v3<dual> xb;
      m3<dual> Rb;
      dual_pose(M.qm + 7 * b, b == beta, comp, xb, Rb);
      v3<dual> tq{dual(0.0), dual(0.0), dual(0.0)};
      int cc = 0;
      for (int j = 0; j < R.nj; ++j) {
        int act = B.joint_act[R.j0 + j];
        if (!act) continue;
        int ja = B.joint_body[2 * (R.j0 + j)], jb = B.joint_body[2 * (R.j0 + j) + 1];
        if ((act == 1 || act == 3) && (ja == b || jb == b)) {
          v3<dual> xa_;
          m3<dual> Ra_;
          dual_pose(M.qm + 7 * ja, ja == beta, comp, xa_, Ra_);
          v3<dual> ax = mul(Ra_, ld3<dual>(B.joint_frame + 18 * (R.j0 + j) + 15));
          double tau = ctrl[R.c0 + cc];
          if (jb == b) tq = tq + ax * tau;
          if (ja == b) tq = tq - ax * tau;
        }
        ++cc;
      }
      dual um[6], uu[6], out[6];
      for (int k = 0; k < 6; ++k) { um[k] = dual(M.um[6 * b + k]); uu[k] = dual(M.u[6 * b + k]); }
      body_terms<dual>(P, M.mass[b], M.inert + 3 * b, Rb, um, uu, tq, out);
      for (int k = 0; k < 6; ++k) s += wu[6 * b + k] * out[k].d;
    }
    // constraint rows and their forces in r_dyn
    const int ng = n_groups(R);
    for (int g = 0; g < ng; ++g) {
      int row = group_row(R, g);
      int a = M.r_a[row], c = M.r_b[row];
      if (a != beta && c != beta) continue;
      int kind = M.r_kind[row];
      if (kind == RK_CONTACT && P.truncate) continue;
      int n = kind == RK_CONTACT ? 3 : 1;
      GroupIn<dual> ind;
      dual_pose(M.qm + 7 * a, a == beta, comp, ind.xa, ind.Ra);
      if (c >= 0) dual_pose(M.qm + 7 * c, c == beta, comp, ind.xb, ind.Rb);
      else {
        ind.xb = v3<dual>{dual(0.0), dual(0.0), dual(0.0)};
        for (int k = 0; k < 9; ++k) ind.Rb.a[k] = dual((k % 4 == 0) ? 1.0 : 0.0);
      }
      dual ua[6], ub[6], lg[3];
      for (int k = 0; k < 6; ++k) {
        ua[k] = dual(M.u[6 * a + k]);
        ub[k] = c >= 0 ? dual(M.u[6 * c + k]) : dual(0.0);
      }
      #pragma unroll
      for (int k = 0; k < 3; ++k) if (k < n) lg[k] = dual(M.lam[row + k]);
      ind.ua = ua;
      ind.ub = c >= 0 ? ub : nullptr;
      ind.lg = lg;
      ind.target = dual(kind == RK_SERVO ? M.sv_in[row - 5 * R.nj] : 0.0);
      if (kind == RK_SERVO && B.joint_act[R.j0 + M.r_idx[row]] == 4)  // theta* - theta(q-), q- seeded
        ind.target.d = -joint_angle_der(ind.Ra, ind.Rb, B.joint_frame + 18 * (R.j0 + M.r_idx[row]));
      if (kind == RK_CONTACT) {
        int ci = M.r_idx[row];
        int s_ = M.c_slot[ci];
        const int* si = B.slot_int + 4 * (R.s0 + s_);
        const double* sr = B.slot_real + 9 * (R.s0 + s_);
        const double* obs = si[0] == 1 ? B.obs_box + 6 * (R.o0 + si[3]) : nullptr;
        Feature F = M.c_feat[ci];
        m3<dual> Rb2 = ind.Rb;
        v3<dual> xb2 = ind.xb;
        if (si[0] != 2) { Rb2 = ind.Ra; xb2 = v3<dual>{dual(0.0), dual(0.0), dual(0.0)}; }
        ind.fr = slot_frame<dual>(si[0], sr, obs, ind.xa, ind.Ra, xb2, Rb2, F, false, nullptr, &R.hm, si[3]);
      }
      dual rd[3], Jd[36];
      double Dd[3];
      eval_row_group<dual, Team::kRim>(B, P, R, M, row, ind, rd, Jd, Dd);
      #pragma unroll
      for (int k = 0; k < 3; ++k) if (k < n) {
        s += wl[row + k] * M.D[row + k] * rd[k].d;
        double jw = 0.0;
        for (int q = 0; q < 6; ++q) jw += Jd[12 * k + q].d * wu[6 * a + q];
        if (c >= 0) for (int q = 0; q < 6; ++q) jw += Jd[12 * k + 6 + q].d * wu[6 * c + q];
        s -= h * M.lam[row + k] * jw;
      }
    }
    // direct term of q+ = q- + h G(q-) u*: x -> identity, quaternion -> (I + h/2 L(w))^T
    const double* gr = M.gq + 7 * beta;
    double direct;
    if (comp < 3) {
      direct = gr[comp];
    } else {
      const double* u = M.u + 6 * beta;
      v3<double> wv{u[3], u[4], u[5]}, gv{gr[3], gr[4], gr[5]};
      v3<double> tv = -cross(wv, gv) - wv * gr[6];
      double tw4 = dot(wv, gv);
      double add = comp == 3 ? tv.x : (comp == 4 ? tv.y : (comp == 5 ? tv.z : tw4));
      direct = gr[comp] + 0.5 * h * add;
    }
    gq_prev[7 * R.b0 + p] = direct + s;
  }
  // model parameters, Eq. (17) with xi a parameter (the FB scales and the
  // Schur regularisation held as in the solve): a body's mass enters its
  // dynamics rows, m (u - u-) - h m g; a servo gain its servo row through
  // lambda / k_p; a friction coefficient the friction rows of its slot's active
  // contact.  Every entry is written once: zero where the parameter does not
  // enter this step.
  if (g_mass)
    for (int b = t.rank(); b < nb; b += t.size()) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += wu[6 * b + k] * ((M.u[6 * b + k] - M.um[6 * b + k]) - h * P.g[k]);
      g_mass[R.b0 + b] = s;
    }
  if (g_kp)
    for (int j = t.rank(); j < R.nj; j += t.size()) {
      double g = 0.0;
      for (int i = 5 * R.nj; i < 5 * R.nj + R.nsv; ++i)
        if (M.r_idx[i] == j) {
          const double kp = B.joint_kp[R.j0 + j];
          if (B.joint_act[R.j0 + j] == 4) {  // d/dk_p of alpha lambda + alpha k_p e = alpha^2 (k_d e - h lambda)
            const double kd = B.joint_kd[R.j0 + j], al = 1.0 / (kd + h * kp);
            const double e = -M.sv_in[i - 5 * R.nj];  // theta(q-) - theta*
            g = wl[i] * M.D[i] * (al * al * (kd * e - h * M.lam[i]));
          } else {
            g = wl[i] * M.D[i] * (-M.lam[i] / (kp * kp));
          }
        }
      g_kp[R.j0 + j] = g;
    }
  if (g_mu)
    for (int s = t.rank(); s < R.ns; s += t.size()) {
      const int c = M.s_act[s];
      double g = 0.0;
      if (c >= 0) {  // d r / d mu of the contact's rows, one dual evaluation with mu seeded
        const int row = 5 * R.nj + R.nsv + 3 * c;
        const int a = M.r_a[row], b = M.r_b[row];
        GroupIn<double> in = group_in_lds(M, row, M.u, M.lam, 0.0);
        dual ua[6], ub[6], lg[3];
        for (int k = 0; k < 6; ++k) {
          ua[k] = dual(M.u[6 * a + k]);
          ub[k] = b >= 0 ? dual(M.u[6 * b + k]) : dual(0.0);
        }
        for (int k = 0; k < 3; ++k) lg[k] = dual(M.lam[row + k]);
        GroupIn<dual> ind;
        ind.xa = v3<dual>{in.xa.x, in.xa.y, in.xa.z};
        ind.xb = v3<dual>{in.xb.x, in.xb.y, in.xb.z};
        for (int k = 0; k < 9; ++k) { ind.Ra.a[k] = in.Ra.a[k]; ind.Rb.a[k] = in.Rb.a[k]; }
        ind.ua = ua;
        ind.ub = b >= 0 ? ub : nullptr;
        ind.lg = lg;
        ind.target = dual(0.0);
        ind.fr = lift_frame(in.fr);
        dual rd[3], Jd[36];
        double Dd[3];
        eval_group<dual, Team::kRim>(B, P, R, RK_CONTACT, M.r_idx[row], M.r_sub[row], b >= 0, M.c_r[c], dual(M.c_mu[c], 1.0),
                         M.c_sn[c], M.c_sf[c], M.c_kind[c], ind, rd, Jd, Dd);
        for (int k = 1; k < 3; ++k) g += wl[row + k] * M.D[row + k] * rd[k].d;
      }
      g_mu[R.s0 + s] = g;
    }
  t.sync();
  return true;
}

}  // namespace ost
