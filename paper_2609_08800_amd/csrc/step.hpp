// Team procedures of the fused per-world step: contact refresh, Newton loop
// with best-iterate selection (Sec. III-C), and the implicit adjoint
// (Sec. III-D) that back-solves the stored Schur factor.
#pragma once

#include "world.hpp"

namespace ost {

// ------------------------------------------------------------ small helpers
OST_HD v3<double> ldv(const double* p) { return v3<double>{p[0], p[1], p[2]}; }
OST_HD m3<double> ldm(const double* p) {
  m3<double> R;
  for (int i = 0; i < 9; ++i) R.a[i] = p[i];
  return R;
}
OST_HD void stv(double* p, const v3<double>& v) { p[0] = v.x; p[1] = v.y; p[2] = v.z; }

struct RowInfo {
  int kind, a, b, idx, sub, g, n;
};

OST_HD int n_groups(const WorldRef& R) { return 5 * R.nj + R.nsv + R.nc; }
OST_HD int group_row(const WorldRef& R, int g) {
  int base = 5 * R.nj + R.nsv;
  return g < base ? g : base + 3 * (g - base);
}

// Input of a group evaluated at (u, lambda) from the LDS copies (double).
OST_HD GroupIn<double> group_in_lds(const WorldMem& M, int row, const double* u, const double* lam, double target) {
  GroupIn<double> in;
  int a = M.r_a[row], b = M.r_b[row];
  in.xa = ldv(M.xm + 3 * a);
  in.Ra = ldm(M.Rm + 9 * a);
  if (b >= 0) {
    in.xb = ldv(M.xm + 3 * b);
    in.Rb = ldm(M.Rm + 9 * b);
  } else {
    in.xb = v3<double>{0, 0, 0};
    for (int i = 0; i < 9; ++i) in.Rb.a[i] = (i % 4 == 0) ? 1.0 : 0.0;
  }
  in.ua = u + 6 * a;
  in.ub = b >= 0 ? u + 6 * b : nullptr;
  in.lg = lam + row;
  in.target = target;
  if (M.r_kind[row] == RK_CONTACT) {
    int c = M.r_idx[row];
    in.fr.n = ldv(M.c_n + 3 * c);
    in.fr.t1 = ldv(M.c_t1 + 3 * c);
    in.fr.t2 = ldv(M.c_t2 + 3 * c);
    in.fr.noff = M.c_noff[c];
    in.fr.la = ldv(M.c_la + 3 * c);
    in.fr.lb = ldv(M.c_lb + 3 * c);
    in.fr.ax = ldv(M.c_ax + 3 * c);
    in.fr.disc = M.c_ax[3 * c] != 0.0 || M.c_ax[3 * c + 1] != 0.0 || M.c_ax[3 * c + 2] != 0.0;
  }
  return in;
}

// Compliance alpha of a servo row (Eq. (8)): 1/k_p for a speed target,
// 1/(k_d + h k_p) for an angle target.
OST_HD double servo_compliance(const Batch& B, const WorldRef& R, int joint, double h) {
  const double kp = B.joint_kp[R.j0 + joint];
  return B.joint_act[R.j0 + joint] == 4 ? 1.0 / (B.joint_kd[R.j0 + joint] + h * kp) : 1.0 / kp;
}

OST_HD double servo_target(const Batch& B, const WorldRef& R, const double* ctrl, int joint);

// The servo row's input for the row evaluation: the target speed (act 2), 0
// (act 3), or theta* - theta(q-) (act 4), which holds for the whole step,
// since the joint angle is taken at q- (Eq. (8)).
OST_HD double servo_input(const Batch& B, const WorldRef& R, const WorldMem& M, const double* ctrl, int joint) {
  const double target = servo_target(B, R, ctrl, joint);
  if (B.joint_act[R.j0 + joint] != 4) return target;
  const int a = B.joint_body[2 * (R.j0 + joint)], b = B.joint_body[2 * (R.j0 + joint) + 1];
  return target - joint_angle(ldm(M.Rm + 9 * a), ldm(M.Rm + 9 * b), B.joint_frame + 18 * (R.j0 + joint));
}

OST_HD double servo_target(const Batch& B, const WorldRef& R, const double* ctrl, int joint) {
  int act = B.joint_act[R.j0 + joint];
  if (act != 2 && act != 4) return 0.0;  // speed (2) or angle (4) from the control; 3: speed 0
  int c = 0;
  for (int j = 0; j < joint; ++j)
    if (B.joint_act[R.j0 + j]) ++c;
  return ctrl[R.c0 + c];
}

template <class T, bool kRim = true>
OST_HD void eval_row_group(const Batch& B, const Params& P, const WorldRef& R, const WorldMem& M, int row,
                           const GroupIn<T>& in, T* r, T* J, double* D) {
  int kind = M.r_kind[row];
  int c = kind == RK_CONTACT ? M.r_idx[row] : 0;
  eval_group<T, kRim>(B, P, R, kind, M.r_idx[row], M.r_sub[row], M.r_b[row] >= 0, kind == RK_CONTACT ? M.c_r[c] : 0.0,
                kind == RK_CONTACT ? M.c_mu[c] : 0.0, kind == RK_CONTACT ? M.c_sn[c] : 1.0,
                kind == RK_CONTACT ? M.c_sf[c] : 1.0, kind == RK_CONTACT ? M.c_kind[c] : 0, in, r, J, D);
}

// --------------------------------------------------------------------------
// Prologue: bodies at q-, contact refresh (A1), rows, warm start, FB scales.
// --------------------------------------------------------------------------
// The slot whose heightmap search a terrain slot s shares: the slot r places
// before it when s takes rank r > 0 of the same body point and radius as that
// rank-0 slot, else s itself.
OST_HD int hm_leader(const Batch& B, const WorldRef& R, int s) {
  const int* si = B.slot_int + 4 * (R.s0 + s);
  const int r = si[3];
  if (r <= 0 || r >= 4 || s - r < 0) return s;
  const int l = s - r;
  const int* li = B.slot_int + 4 * (R.s0 + l);
  const double* sr = B.slot_real + 9 * (R.s0 + s);
  const double* lr = B.slot_real + 9 * (R.s0 + l);
  if (li[0] != 3 || li[3] != 0 || li[1] != si[1]) return s;
  for (int k = 0; k < 4; ++k)
    if (!(lr[k] == sr[k])) return s;
  return l;
}

OST_HD double ll_bits(long long v) {
  double d;
  memcpy(&d, &v, sizeof d);
  return d;
}
OST_HD long long bits_ll(double d) {
  long long v;
  memcpy(&v, &d, sizeof v);
  return v;
}

// Heightmap candidates of the world's terrain slots at q- (the choice of
// hm_select, computed together): one search per searching slot (hm_leader),
// its cells spread over the team, each thread keeping the best four of its
// cells; the lists are merged in the candidates' order, so the chosen keys do
// not depend on the split.  The best four keys of searching slot l are left
// in A[4 l .. 4 l + 3] (the Schur matrix's storage is free until assembly; a
// world row capacity's square of it is always there), the searching slots in
// s_act.  Returns false, with nothing done, when the world has no heightmap
// or too little room, and each slot then searches for itself.
template <class Team>
OST_HD bool terrain_candidates(Team& t, const Batch& B, const Params& P, const WorldRef& R, const WorldMem& M) {
  if (R.hm.n < 2) return false;
  const size_t room = M.a_room;  // the Schur matrix's storage in this carve
  if (t.rank() == 0) {
    int n = 0;
    for (int s = 0; s < R.ns; ++s)
      if (B.slot_int[4 * (R.s0 + s)] == 3 && hm_leader(B, R, s) == s) M.s_act[n++] = s;
    M.iscal[9] = n;
  }
  t.sync();
  const int ntask = M.iscal[9];
  if (ntask == 0 || room < (size_t)4 * R.ns + (size_t)8 * ntask) {
    t.sync();
    return false;
  }
  double* fin = M.A;
  double* lists = M.A + 4 * R.ns;
  int G = t.size() / ntask;
  const int gmax = (int)((room - (size_t)4 * R.ns) / ((size_t)8 * ntask));
  if (G > gmax) G = gmax;
  if (G < 1) G = 1;
  for (int u = t.rank(); u < ntask * G; u += t.size()) {
    const int task = u / G, part = u - task * G, s = M.s_act[task];
    const int* si = B.slot_int + 4 * (R.s0 + s);
    const double* sr = B.slot_real + 9 * (R.s0 + s);
    const int a = si[1];
    // the proxy centre and search radius of the slot loop below
    const v3<double> la = mul(ldm(M.Rm + 9 * a), ldv(sr));
    const double* ua = M.um + 6 * a;
    const v3<double> vp = ldv(ua) + cross(ldv(ua + 3), la);
    const double rc = sr[3] + P.d0 + P.h * ::sqrt(dot(vp, vp));
    const v3<double> Pc = ldv(M.xm + 3 * a) + la;
    long long bd[4];
    int bk[4];
    const int nb = hm_best4(R.hm, Pc, rc, part, G, bd, bk);
    double* o = lists + 8 * u;
    for (int q = 0; q < 4; ++q) {
      o[q] = q < nb ? ll_bits(bd[q]) : 0.0;
      o[4 + q] = q < nb ? (double)bk[q] : -1.0;
    }
  }
  t.sync();
  for (int task = t.rank(); task < ntask; task += t.size()) {
    long long bd[4];
    int bk[4], nb = 0;
    for (int part = 0; part < G; ++part) {
      const double* o = lists + 8 * (task * G + part);
      for (int q = 0; q < 4 && o[4 + q] >= 0.0; ++q) hm_insert(bd, bk, nb, bits_ll(o[q]), (int)o[4 + q]);
    }
    double* f = fin + 4 * M.s_act[task];
    for (int q = 0; q < 4; ++q) f[q] = q < nb ? (double)bk[q] : -1.0;
  }
  t.sync();
  return true;
}

// Returns false, with only the workspace touched, when the world's active
// contacts exceed the carve's contact capacity (M.nc_cap): the launch then
// hands the world to one whose workspace holds them.
// Activation test of the contact refresh: the slot's gap at q- plus one step
// of its approach speed along the normal (relative velocity of the contact
// point) within delta0.  ub is body b's velocity for a body-face slot.
OST_HD bool approach_active(const Params& P, int kind, const double* sr, const Frame<double>& C, double gap,
                            const v3<double>& xa, const double* ua, const v3<double>& xb, const double* ub) {
  v3<double> d = C.n;  // from the proxy's contact point to its centre
  if (C.disc) rim_depth(C.n, C.ax, sr[3], &d);
  v3<double> pc = xa + C.la - d * sr[3];
  v3<double> vr = ldv(ua) + cross(ldv(ua + 3), pc - xa);
  if (kind == 2) vr = vr - (ldv(ub) + cross(ldv(ub + 3), pc - xb));
  double vn = dot(C.n, vr);
  return gap + P.h * (vn < 0.0 ? vn : 0.0) <= P.d0;
}

// Active contacts of world R at q- by the refresh's test, for a launch plan:
// slots s0, s0 + ds, ... of the world (a team's share), terrain slots left
// out (their mesh search is the step's) and counted in *n_terrain.  Returns
// the share's count of the other slots.
OST_HD int count_active(const Batch& B, const Params& P, const WorldRef& R, const double* q_prev,
                        const double* u_prev, int s0, int ds, int* n_terrain) {
  int n = 0;
  *n_terrain = 0;
  for (int s = s0; s < R.ns; s += ds) {
    const int* si = B.slot_int + 4 * (R.s0 + s);
    const double* sr = B.slot_real + 9 * (R.s0 + s);
    const int kind = si[0], a = si[1], b = si[2];
    if (kind == 3) {
      ++*n_terrain;
      continue;
    }
    const double* qa = q_prev + 7 * (R.b0 + a);
    const v3<double> xa = ldv(qa);
    const m3<double> Ra = quat_to_R(qa[3], qa[4], qa[5], qa[6]);
    v3<double> xb{0, 0, 0};
    m3<double> Rb = Ra;
    if (kind == 2) {
      const double* qb = q_prev + 7 * (R.b0 + b);
      xb = ldv(qb);
      Rb = quat_to_R(qb[3], qb[4], qb[5], qb[6]);
    }
    const double* obs = kind == 1 ? B.obs_box + 6 * (R.o0 + si[3]) : nullptr;
    Feature F{};
    double gap;
    Frame<double> C = slot_frame<double>(kind, sr, obs, xa, Ra, xb, Rb, F, true, &gap, &R.hm, si[3], 0.0, false);
    n += approach_active(P, kind, sr, C, gap, xa, u_prev + 6 * (R.b0 + a), xb,
                         kind == 2 ? u_prev + 6 * (R.b0 + b) : nullptr);
  }
  return n;
}

template <class Team>
OST_HD bool prologue(Team& t, const Batch& B, const Params& P, WorldRef& R, const double* q_prev,
                     const double* u_prev, const double* ctrl, const double* lam_prev, WorldMem& M) {
  const int nb = R.nb;
  for (int b = t.rank(); b < nb; b += t.size()) {
    const double* q = q_prev + 7 * (R.b0 + b);
    const double* u = u_prev + 6 * (R.b0 + b);
    for (int k = 0; k < 7; ++k) M.qm[7 * b + k] = q[k];
    for (int k = 0; k < 6; ++k) { M.um[6 * b + k] = u[k]; M.u[6 * b + k] = u[k]; }
    for (int k = 0; k < 3; ++k) M.xm[3 * b + k] = q[k];
    m3<double> Rm = quat_to_R(q[3], q[4], q[5], q[6]);
    for (int k = 0; k < 9; ++k) M.Rm[9 * b + k] = Rm.a[k];
    const double* I = B.body_inertia + 3 * (R.b0 + b);
    M.mass[b] = B.body_mass[R.b0 + b];
    for (int k = 0; k < 3; ++k) M.inert[3 * b + k] = I[k];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = 0.0, si = 0.0;
        for (int k = 0; k < 3; ++k) {
          s += Rm.a[3 * i + k] * I[k] * Rm.a[3 * j + k];
          si += Rm.a[3 * i + k] / I[k] * Rm.a[3 * j + k];
        }
        M.Iw[9 * b + 3 * i + j] = s;
        M.Iwi[9 * b + 3 * i + j] = si;
      }
    for (int k = 0; k < 6; ++k) M.fext[6 * b + k] = 0.0;  // actuator torque (angular part)
  }
  t.sync();
  if (t.rank() == 0) {  // actuator torques about the joint axis at q-
    int c = 0;
    for (int j = 0; j < R.nj; ++j) {
      int act = B.joint_act[R.j0 + j];
      if (!act) continue;
      if (act == 1 || act == 3) {
        int a = B.joint_body[2 * (R.j0 + j)], b = B.joint_body[2 * (R.j0 + j) + 1];
        v3<double> ax = mul(ldm(M.Rm + 9 * a), ldv(B.joint_frame + 18 * (R.j0 + j) + 15));
        double tau = ctrl[R.c0 + c];
        for (int k = 0; k < 3; ++k) {
          M.fext[6 * b + 3 + k] += tau * at(ax, k);
          M.fext[6 * a + 3 + k] -= tau * at(ax, k);
        }
      }
      ++c;
    }
  }
  // contact refresh: frame and activation of every slot at q-
  const bool keyed = terrain_candidates(t, B, P, R, M);
  for (int s = t.rank(); s < R.ns; s += t.size()) {
    const int* si = B.slot_int + 4 * (R.s0 + s);
    const double* sr = B.slot_real + 9 * (R.s0 + s);
    int kind = si[0], a = si[1], b = si[2];
    Feature F{};
    double gap;
    if (kind == 3 && keyed) F.hkey = si[3] >= 0 && si[3] < 4 ? (int)M.A[4 * hm_leader(B, R, s) + si[3]] : -1;
    v3<double> xb{0, 0, 0};
    m3<double> Rb = ldm(M.Rm + 9 * a);
    if (kind == 2) { xb = ldv(M.xm + 3 * b); Rb = ldm(M.Rm + 9 * b); }
    const double* obs = kind == 1 ? B.obs_box + 6 * (R.o0 + si[3]) : nullptr;
    double rc = 0.0;
    if (kind == 3) {  // search radius: proxy radius, margin and one step at the proxy centre's speed
      const double* ua = M.um + 6 * a;
      v3<double> la = mul(ldm(M.Rm + 9 * a), ldv(sr));
      v3<double> vp = ldv(ua) + cross(ldv(ua + 3), la);
      rc = sr[3] + P.d0 + P.h * ::sqrt(dot(vp, vp));
    }
    Frame<double> C = slot_frame<double>(kind, sr, obs, ldv(M.xm + 3 * a), ldm(M.Rm + 9 * a), xb, Rb, F, true, &gap,
                                         &R.hm, si[3], rc, kind == 3 && keyed);
    M.s_act[s] = approach_active(P, kind, sr, C, gap, ldv(M.xm + 3 * a), M.um + 6 * a, xb,
                                 kind == 2 ? M.um + 6 * b : nullptr) ? 1 : 0;
    M.s_feat[s] = F;
  }
  t.sync();
  if (t.rank() == 0) {  // ascending-slot compaction, at most contact_cap; s_act becomes the position or -1
    int nc = 0, of = 0, na = 0;
    for (int s = 0; s < R.ns; ++s) na += M.s_act[s];
    M.iscal[10] = (na < R.cap ? na : R.cap) > M.nc_cap;
    for (int s = 0; s < R.ns && !M.iscal[10]; ++s)
      if (M.s_act[s]) {
        if (nc < R.cap) {
          M.c_slot[nc] = s;
          M.s_act[s] = nc++;
        } else {
          of = 1;
          M.s_act[s] = -1;
        }
      } else {
        M.s_act[s] = -1;
      }
    M.iscal[0] = nc;
    M.iscal[1] = of;
  }
  t.sync();
  if (M.iscal[10]) return false;
  R.nc = M.iscal[0];
  R.m = 5 * R.nj + R.nsv + 3 * R.nc;
  for (int c = t.rank(); c < R.nc; c += t.size()) {
    int s = M.c_slot[c];
    const int* si = B.slot_int + 4 * (R.s0 + s);
    const double* sr = B.slot_real + 9 * (R.s0 + s);
    int kind = si[0], a = si[1], b = si[2];
    Feature F = M.s_feat[s];
    v3<double> xb{0, 0, 0};
    m3<double> Rb = ldm(M.Rm + 9 * a);
    if (kind == 2) { xb = ldv(M.xm + 3 * b); Rb = ldm(M.Rm + 9 * b); }
    const double* obs = kind == 1 ? B.obs_box + 6 * (R.o0 + si[3]) : nullptr;
    Frame<double> C = slot_frame<double>(kind, sr, obs, ldv(M.xm + 3 * a), ldm(M.Rm + 9 * a), xb, Rb, F, false, nullptr,
                                         &R.hm, si[3]);
    M.c_feat[c] = F;
    M.c_kind[c] = kind;
    M.c_a[c] = a;
    M.c_b[c] = kind == 2 ? b : -1;
    M.c_r[c] = sr[3];
    M.c_mu[c] = sr[4];
    stv(M.c_n + 3 * c, C.n);
    stv(M.c_t1 + 3 * c, C.t1);
    stv(M.c_t2 + 3 * c, C.t2);
    M.c_noff[c] = C.noff;
    stv(M.c_la + 3 * c, C.la);
    stv(M.c_lb + 3 * c, C.lb);
    stv(M.c_ax + 3 * c, C.ax);
    M.c_sn[c] = 1.0;
    M.c_sf[c] = 1.0;
  }
  // row layout: [5 per revolute joint][servo rows][3 per active contact]
  const int base = 5 * R.nj + R.nsv;
  for (int i = t.rank(); i < R.m; i += t.size()) {
    int kind, a, b, idx, sub, g, lslot;
    if (i < 5 * R.nj) {
      idx = i / 5;
      sub = i % 5;
      kind = sub < 3 ? RK_ANCHOR : RK_AXIS;
      if (sub >= 3) sub -= 3;
      a = B.joint_body[2 * (R.j0 + idx)];
      b = B.joint_body[2 * (R.j0 + idx) + 1];
      g = i;
      lslot = i;
    } else if (i < base) {
      int sv = i - 5 * R.nj, c = -1;
      idx = 0;
      for (int j = 0; j < R.nj; ++j) {
        int act = B.joint_act[R.j0 + j];
        if (act == 2 || act == 3 || act == 4) {
          if (++c == sv) { idx = j; break; }
        }
      }
      kind = RK_SERVO;
      sub = 0;
      a = B.joint_body[2 * (R.j0 + idx)];
      b = B.joint_body[2 * (R.j0 + idx) + 1];
      g = i;
      lslot = i;
    } else {
      int c = (i - base) / 3;
      sub = (i - base) % 3;
      kind = RK_CONTACT;
      idx = c;
      int s = M.c_slot[c];
      const int* si = B.slot_int + 4 * (R.s0 + s);
      a = si[1];
      b = si[0] == 2 ? si[2] : -1;
      g = base + 3 * c;
      lslot = base + 3 * s + sub;
    }
    M.r_kind[i] = kind;
    M.r_a[i] = a;
    M.r_b[i] = b;
    M.r_idx[i] = idx;
    M.r_sub[i] = sub;
    M.r_g[i] = g;
    M.lam[i] = lam_prev ? lam_prev[R.l0 + lslot] : 0.0;
  }
  t.sync();
  // Band of the Schur matrix: entry (i, j) is structurally non-zero only if
  // rows i and j act on a common body, so rows couple back to the first row
  // that touches one of their bodies.
  for (int b = t.rank(); b < nb; b += t.size()) {
    int f = R.m;
    for (int i = 0; i < R.m; ++i)
      if (M.r_a[i] == b || M.r_b[i] == b) { f = i; break; }
    M.b_first[b] = f;
  }
  t.sync();
  int bw = 0;
  for (int i = t.rank(); i < R.m; i += t.size()) {
    int f = M.b_first[M.r_a[i]];
    if (M.r_b[i] >= 0 && M.b_first[M.r_b[i]] < f) f = M.b_first[M.r_b[i]];
    if (i - f > bw) bw = i - f;
  }
  R.bw = t.imax(bw, M.red);
  if (t.rank() == 0) M.iscal[3] = R.bw;
  // servo inputs: the target speed, or the angle error theta* - theta(q-)
  for (int s = t.rank(); s < R.nsv; s += t.size()) M.sv_in[s] = servo_input(B, R, M, ctrl, M.r_idx[5 * R.nj + s]);
  t.sync();
  return true;
}

// Clamp of the friction multipliers to the Coulomb disk of radius
// max(mu lambda_n, delta_g) (Sec. III-B safeguard).
template <class Team> OST_HD void clamp_all(Team& t, const Params& P, const WorldRef& R, const WorldMem& M, double* lam) {
  const int base = 5 * R.nj + R.nsv;
  for (int c = t.rank(); c < R.nc; c += t.size()) {
    int i = base + 3 * c;
    double lim = M.c_mu[c] * lam[i];
    if (lim < P.dg) lim = P.dg;
    double n = ::sqrt(lam[i + 1] * lam[i + 1] + lam[i + 2] * lam[i + 2]);
    if (n > lim) {
      double s = n > 0.0 ? lim / n : 0.0;
      lam[i + 1] *= s;
      lam[i + 2] *= s;
    }
  }
  t.sync();
}

// M~^-1 applied to a 6-vector of body b.
OST_HD void minv6(const WorldMem& M, int b, const double* x, double* y) {
  double im = 1.0 / M.mass[b];
  y[0] = x[0] * im; y[1] = x[1] * im; y[2] = x[2] * im;
  const double* Ii = M.Iwi + 9 * b;
  for (int i = 0; i < 3; ++i) y[3 + i] = Ii[3 * i] * x[3] + Ii[3 * i + 1] * x[4] + Ii[3 * i + 2] * x[5];
}

// --------------------------------------------------------------------------
// Residual at (u, lam): J, raw rows, r_dyn, norm; with want_G also the
// generalized Jacobian of the scaled rows (Y = G_u M~^-1, G_lambda) and the
// Delassus diagonal.  Returns the residual norm.
// --------------------------------------------------------------------------
template <class Team>
OST_HD double evaluate(Team& t, const Batch& B, const Params& P, const WorldRef& R, const WorldMem& M,
                       const double* ctrl, const double* u, const double* lam, bool want_G) {
  const int ng = n_groups(R);
  for (int g = t.rank(); g < ng; g += t.size()) {
    int row = group_row(R, g);
    int kind = M.r_kind[row];
    int n = kind == RK_CONTACT ? 3 : 1;
    double target = kind == RK_SERVO ? M.sv_in[row - 5 * R.nj] : 0.0;
    GroupIn<double> in = group_in_lds(M, row, u, lam, target);
    double r[3], D[3];
    double* Jg = M.J + 12 * row;
    eval_row_group<double, Team::kRim>(B, P, R, M, row, in, r, Jg, D);
    #pragma unroll
    for (int k = 0; k < 3; ++k) if (k < n) {
      M.res[row + k] = r[k];
      M.D[row + k] = D[k];
    }
    if (!want_G) continue;
    int a = M.r_a[row], b = M.r_b[row];
    // the generalized Jacobian goes straight to the workspace: G_u into the rows
    // of Y (turned into Y = G_u M~^-1 in place below), G_lambda into Gl
    double* Gu = M.Y + 12 * row;
    double* Gl = M.Gl + 3 * row;
    if (kind == RK_CONTACT) {
      int c = M.r_idx[row];
      contact_G<Team::kRim>(P, in, b >= 0, M.c_r[c], M.c_mu[c], M.c_sn[c], M.c_sf[c], M.c_kind[c], Jg, D, Gu, Gl);
    } else {  // joint rows: D r = c(q(u)) / h, so D dr/du = J; servo rows: dr/du = J, dr/dlambda = alpha
      for (int q = 0; q < 12; ++q) Gu[q] = Jg[q];
      Gl[0] = kind == RK_SERVO ? servo_compliance(B, R, M.r_idx[row], P.h) : 0.0;
      Gl[1] = 0.0;
      Gl[2] = 0.0;
    }
    #pragma unroll
    for (int k = 0; k < 3; ++k) if (k < n) {
      double* Y = M.Y + 12 * (row + k);
      double g[12];
      for (int q = 0; q < 12; ++q) g[q] = Y[q];
      minv6(M, a, g, Y);
      if (b >= 0) minv6(M, b, g + 6, Y + 6);
      else for (int q = 6; q < 12; ++q) Y[q] = 0.0;
      const double* Jr = Jg + 12 * k;
      double MJ[12], s = 0.0;
      minv6(M, a, Jr, MJ);
      for (int q = 0; q < 6; ++q) s += Jr[q] * MJ[q];
      if (b >= 0) {
        minv6(M, b, Jr + 6, MJ + 6);
        for (int q = 6; q < 12; ++q) s += Jr[q] * MJ[q];
      }
      M.Abar[row + k] = s;
    }
  }
  t.sync();
  // r_dyn per (body, component); constraint forces summed over rows in order
  for (int e = t.rank(); e < 6 * R.nb; e += t.size()) {
    int b = e / 6, comp = e - 6 * b;
    double out[6];
    v3<double> tq{M.fext[6 * b + 3], M.fext[6 * b + 4], M.fext[6 * b + 5]};
    body_terms<double>(P, M.mass[b], M.inert + 3 * b, ldm(M.Rm + 9 * b), M.um + 6 * b, u + 6 * b, tq, out);
    double v = out[comp];
    const int m = R.m;
    for (int i0 = 0; i0 < m; i0 += 4) {  // rows in fours: the loads first, then the sum in row order
      int ra[4], rb[4];
      double ja[4], jb[4], lm[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + r < m ? i0 + r : m - 1;
        ra[r] = i0 + r < m ? M.r_a[i] : -2;
        rb[r] = i0 + r < m ? M.r_b[i] : -2;
        ja[r] = M.J[12 * i + comp];
        jb[r] = M.J[12 * i + 6 + comp];
        lm[r] = lam[i];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (ra[r] == b) v -= P.h * (ja[r] * lm[r]);
        if (rb[r] == b) v -= P.h * (jb[r] * lm[r]);
      }
    }
    M.rdyn[e] = v;
  }
  t.sync();
  // sum of squares over a fixed partition into 64 lanes, so the value does not
  // depend on the team size
  double s = 0.0;
  int ntot = 6 * R.nb + R.m;
  for (int l = t.rank(); l < 64; l += t.size())
    for (int i = l; i < ntot; i += 64) {
      double v = i < 6 * R.nb ? M.rdyn[i] : M.res[i - 6 * R.nb];
      s += v * v;
    }
  return ::sqrt(t.sum64(s, M.red));
}

// Schur matrix of Eq. (12) with the generalized Jacobian: A = G_u M~^-1 J^T
// + G_lambda / h + dreg diag(J M~^-1 J^T), and its right-hand side.
template <class Team>
OST_HD void assemble(Team& t, const Params& P, const WorldRef& R, const WorldMem& M, double dreg, bool with_rhs) {
  const int m = R.m, bw = R.bw, wd = 2 * bw + 1, ld = lda(m);
  const bool dense = wd >= m;
  const double ih = 1.0 / P.h;
  const int n_e = dense ? m * m : m * wd;
  for (int e = t.rank(); e < n_e; e += t.size()) {
    int i, j;
    if (dense) { i = e / m; j = e - i * m; }
    else {
      i = e / wd;
      j = i - bw + (e - i * wd);
      if (j < 0 || j >= m) continue;
    }
    // all loads of the entry at once, then the sums of the shared bodies' blocks in order
    double Y[12], Jj[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) { Y[k] = M.Y[12 * i + k]; Jj[k] = M.J[12 * j + k]; }
    int ai = M.r_a[i], bi = M.r_b[i], aj = M.r_a[j], bj = M.r_b[j];
    double s = 0.0;
    if (ai == aj) for (int k = 0; k < 6; ++k) s += Y[k] * Jj[k];
    if (ai == bj) for (int k = 0; k < 6; ++k) s += Y[k] * Jj[6 + k];
    if (bi >= 0 && bi == aj) for (int k = 0; k < 6; ++k) s += Y[6 + k] * Jj[k];
    if (bi >= 0 && bi == bj) for (int k = 0; k < 6; ++k) s += Y[6 + k] * Jj[6 + k];
    int gi = M.r_g[i];
    if (M.r_g[j] == gi) s += M.Gl[3 * i + (j - gi)] * ih;
    if (i == j) s += dreg * M.Abar[i];
    M.A[i * ld + j] = s;
  }
  if (with_rhs)
    for (int i = t.rank(); i < m; i += t.size()) {
      const double* Y = M.Y + 12 * i;
      int a = M.r_a[i], b = M.r_b[i];
      double s = 0.0;
      for (int k = 0; k < 6; ++k) s += Y[k] * M.rdyn[6 * a + k];
      if (b >= 0) for (int k = 0; k < 6; ++k) s += Y[6 + k] * M.rdyn[6 * b + k];
      M.rhs[i] = (s - M.D[i] * M.res[i]) * ih;
    }
  t.sync();
}

// Right-hand side of the Schur system alone, rhs = (Y r_dyn - D r_con) / h
// (Eq. (12)), for the matrix-free Newton step.
template <class Team>
OST_HD void schur_rhs(Team& t, const Params& P, const WorldRef& R, const WorldMem& M) {
  const double ih = 1.0 / P.h;
  for (int i = t.rank(); i < R.m; i += t.size()) {
    const double* Y = M.Y + 12 * i;
    int a = M.r_a[i], b = M.r_b[i];
    double s = 0.0;
    for (int k = 0; k < 6; ++k) s += Y[k] * M.rdyn[6 * a + k];
    if (b >= 0) for (int k = 0; k < 6; ++k) s += Y[6 + k] * M.rdyn[6 * b + k];
    M.rhs[i] = (s - M.D[i] * M.res[i]) * ih;
  }
  t.sync();
}

constexpr int kMaxRows = 384;  // largest row count of a world (six rows per lane of a wavefront)

// In-place LU without pivoting, restricted to the band |i - j| <= bw (no
// fill-in leaves the band without pivoting); false on a non-finite pivot or
// one below 1e-14 of its row's largest entry.  One wavefront factors, each
// lane updating its own rows in rounds of eight entries (all loads of a round
// first), so the per-pivot work costs no workgroup barrier; the row maxima
// needed by the pivot test are kept as the rows are updated.
template <class Team> OST_HD bool lu_factor(Team& t, const WorldRef& R, const WorldMem& M) {
  const int m = R.m, bw = R.bw, W = t.wsize(), ld = lda(m);
  double* A = M.A;
  double* rmax = M.rmax;
  if (t.rank() < W) {
    const int lane = t.rank();
    for (int i = lane; i < m; i += W) {  // row maxima of the assembled band
      const int lo = i - bw > 0 ? i - bw : 0, hi = i + bw + 1 < m ? i + bw + 1 : m;
      double v = 0.0;
      for (int j = lo; j < hi; ++j) v = fmax(v, fabs(A[i * ld + j]));
      rmax[i] = v;
    }
    t.wsync();
    int ok = 1;
    for (int k = 0; k < m; ++k) {
      const int hi = k + bw + 1 < m ? k + bw + 1 : m;
      // the lane's first row below the pivot: its column-k entry is read with the pivot
      const int i1 = k + 1 + (lane + W - (k + 1) % W) % W;
      const double piv = A[k * ld + k], rk = rmax[k], a1 = i1 < hi ? A[i1 * ld + k] : 0.0;
      if (!(isfinite(piv) && fabs(piv) > 1e-14 * rk && rk > 0.0)) {
        ok = 0;
        break;
      }
      const double ip = 1.0 / piv;
      const double* Ak = A + k * ld;
      for (int i = i1; i < hi; i += W) {
        double* Ai = A + i * ld;
        const double l = (i == i1 ? a1 : Ai[k]) * ip;
        Ai[k] = l;
        double v = 0.0;
        int j = k + 1;
        for (; j + 7 < hi; j += 8) {  // rounds of eight: all loads first
          double a[8], b[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) { a[q] = Ai[j + q]; b[q] = Ak[j + q]; }
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            a[q] = a[q] - l * b[q];
            Ai[j + q] = a[q];
            v = fmax(v, fabs(a[q]));
          }
        }
        if (j + 3 < hi) {  // a round of four
          double a[4], b[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) { a[q] = Ai[j + q]; b[q] = Ak[j + q]; }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            a[q] = a[q] - l * b[q];
            Ai[j + q] = a[q];
            v = fmax(v, fabs(a[q]));
          }
          j += 4;
        }
        for (; j < hi; ++j) {
          const double a = Ai[j] - l * Ak[j];
          Ai[j] = a;
          v = fmax(v, fabs(a));
        }
        const int hi_i = i + bw + 1 < m ? i + bw + 1 : m;  // entries of the row this pivot leaves alone
        for (; j < hi_i; ++j) v = fmax(v, fabs(Ai[j]));
        rmax[i] = v;
      }
      t.wsync();
    }
    if (lane == 0) M.iscal[2] = ok;
  }
  t.sync();
  return M.iscal[2] != 0;
}

// Solve A x = b (trans = false) or A^T x = b (trans = true) with the banded LU
// in M.A, by one wavefront.  Up to 128 rows, lane l keeps x_l and x_{l+64} in
// registers and takes x_k from its owner lane at step k, with the matrix
// entries of four steps loaded ahead; beyond, x stays in LDS and each segment
// between wavefront syncs writes an entry from one lane and reads it from none.
template <class Team> OST_HD void lu_solve(Team& t, const WorldRef& R, const WorldMem& M, double* x, bool trans) {
  const int m = R.m, bw = R.bw, W = t.wsize(), ld = lda(m);
  const double* A = M.A;
  if (t.rank() < W) {
    const int lane = t.rank();
    if (W == 64 && m <= 128) {
      const int i0 = lane, i1 = lane + 64;
      double x0 = i0 < m ? x[i0] : 0.0, x1 = i1 < m ? x[i1] : 0.0;
      auto get = [&](int k) { return k < 64 ? t.bcast(x0, k) : t.bcast(x1, k - 64); };
      // entry (row i, step k) of the operator: L or U by rows (plain) or by columns (transposed)
      auto ent = [&](int i, int k) { return trans ? A[k * ld + i] : A[i * ld + k]; };
      if (!trans) {
        for (int k0 = 0; k0 < m; k0 += 4) {  // L y = b (unit lower)
          double e0[4], e1[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int k = k0 + q, hi = k + bw + 1 < m ? k + bw + 1 : m;
            e0[q] = (k < m && i0 > k && i0 < hi) ? ent(i0, k) : 0.0;
            e1[q] = (k < m && i1 > k && i1 < hi) ? ent(i1, k) : 0.0;
          }
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (k0 + q < m) {
              const double yk = get(k0 + q);
              x0 -= e0[q] * yk;
              x1 -= e1[q] * yk;
            }
        }
        for (int k0 = m - 1; k0 >= 0; k0 -= 4) {  // U x = y
          double e0[4], e1[4], d[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int k = k0 - q, lo = k - bw > 0 ? k - bw : 0;
            d[q] = k >= 0 ? A[k * ld + k] : 1.0;
            e0[q] = (k >= 0 && i0 >= lo && i0 < k) ? ent(i0, k) : 0.0;
            e1[q] = (k >= 0 && i1 >= lo && i1 < k) ? ent(i1, k) : 0.0;
          }
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (k0 - q >= 0) {
              const int k = k0 - q;
              const double xk = get(k) / d[q];
              if (i0 == k) x0 = xk;
              if (i1 == k) x1 = xk;
              x0 -= e0[q] * xk;
              x1 -= e1[q] * xk;
            }
        }
      } else {
        for (int k0 = 0; k0 < m; k0 += 4) {  // U^T z = b
          double e0[4], e1[4], d[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int k = k0 + q, hi = k + bw + 1 < m ? k + bw + 1 : m;
            d[q] = k < m ? A[k * ld + k] : 1.0;
            e0[q] = (k < m && i0 > k && i0 < hi) ? ent(i0, k) : 0.0;
            e1[q] = (k < m && i1 > k && i1 < hi) ? ent(i1, k) : 0.0;
          }
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (k0 + q < m) {
              const int k = k0 + q;
              const double zk = get(k) / d[q];
              if (i0 == k) x0 = zk;
              if (i1 == k) x1 = zk;
              x0 -= e0[q] * zk;
              x1 -= e1[q] * zk;
            }
        }
        for (int k0 = m - 1; k0 >= 0; k0 -= 4) {  // L^T x = z (unit)
          double e0[4], e1[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int k = k0 - q, lo = k - bw > 0 ? k - bw : 0;
            e0[q] = (k >= 0 && i0 >= lo && i0 < k) ? ent(i0, k) : 0.0;
            e1[q] = (k >= 0 && i1 >= lo && i1 < k) ? ent(i1, k) : 0.0;
          }
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (k0 - q >= 0) {
              const double xk = get(k0 - q);
              x0 -= e0[q] * xk;
              x1 -= e1[q] * xk;
            }
        }
      }
      if (i0 < m) x[i0] = x0;
      if (i1 < m) x[i1] = x1;
    } else if (!trans) {
      for (int k = 0; k < m; ++k) {  // L y = b (unit lower)
        const double yk = x[k];
        const int hi = k + bw + 1 < m ? k + bw + 1 : m;
        for (int i = k + 1 + lane; i < hi; i += W) x[i] -= A[i * ld + k] * yk;
        t.wsync();
      }
      for (int k = m - 1; k >= 0; --k) {  // U x = y
        const double xk = x[k] / A[k * ld + k];
        t.wsync();
        if (lane == k % W) x[k] = xk;
        for (int i = (k - bw > 0 ? k - bw : 0) + lane; i < k; i += W) x[i] -= A[i * ld + k] * xk;
        t.wsync();
      }
    } else {
      for (int k = 0; k < m; ++k) {  // U^T z = b
        const double zk = x[k] / A[k * ld + k];
        const int hi = k + bw + 1 < m ? k + bw + 1 : m;
        t.wsync();
        if (lane == k % W) x[k] = zk;
        for (int i = k + 1 + lane; i < hi; i += W) x[i] -= A[k * ld + i] * zk;
        t.wsync();
      }
      for (int k = m - 1; k >= 0; --k) {  // L^T x = z (unit)
        const double xk = x[k];
        for (int i = (k - bw > 0 ? k - bw : 0) + lane; i < k; i += W) x[i] -= A[k * ld + i] * xk;
        t.wsync();
      }
    }
  }
  t.sync();
}

// Assemble and factor with the regularisation dreg0 (relative to the Delassus
// diagonal), raised tenfold on failure.
template <class Team>
OST_HD bool factor(Team& t, const Params& P, const WorldRef& R, const WorldMem& M, bool with_rhs, double dreg0,
                   double* dreg_used, int* status) {
  double dreg = dreg0;
  for (int attempt = 0; attempt < 8; ++attempt) {
    assemble(t, P, R, M, dreg, with_rhs && attempt == 0);
    if (lu_factor(t, R, M)) {
      *dreg_used = dreg;
      return true;
    }
    *status |= ST_REGULARIZED;
    dreg *= 10.0;
  }
  return false;
}

}  // namespace ost
