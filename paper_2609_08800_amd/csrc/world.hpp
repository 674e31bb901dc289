// One world's backward-Euler step and its adjoint, written for a team of
// threads that share an LDS workspace (one workgroup per world on the GPU).
//
// Team interface: rank(), size(), sync().  Work loops are strided by the team
// size; every reduction runs in a fixed order so results do not depend on
// scheduling (rollout recomputation is bitwise repeatable).
#pragma once

#include "model.hpp"

namespace ost {

// Capacities of one launch (maxima over the batch) and the LDS carve-out.
struct Caps {
  int nb, nj, ns, nc, mr, nsv;
};

struct WorldMem {
  // bodies
  double *xm, *qm, *Rm, *Iw, *Iwi, *mass, *inert, *fext, *um, *u, *du, *rdyn, *ubest, *ut, *gq, *kg;
  // contacts
  int *c_slot, *c_kind, *c_a, *c_b;
  Feature* c_feat;
  double *c_n, *c_t1, *c_t2, *c_noff, *c_la, *c_lb, *c_r, *c_mu, *c_sn, *c_sf;
  double* c_ax;  // rim circles: world axis at q- (zero for a sphere or point proxy)
  // rows
  int *r_kind, *r_a, *r_b, *r_idx, *r_sub, *r_g;
  double *J, *Y, *Gl, *D, *res, *lam, *dlam, *lamt, *lambest, *Abar, *rmax;
  // Schur matrix and right-hand side
  double *A, *rhs;
  // per servo row: its input for the row evaluation (fixed for the step)
  double* sv_in;
  // slot scratch; first row touching each body (band of the Schur matrix)
  int* s_act;
  int* b_first;
  Feature* s_feat;
  // adjoint only: Krylov basis, iterate, Hessenberg matrix, rotations and
  // reduced right-hand side of the refinement solve (null in the forward)
  double *kv, *kx, *kh, *kcs, *ksn, *kgv, *ky;
  // reduction scratch and scalars
  double* red;
  int* iscal;
  double* dscal;
  // capacities of this carve: doubles at A, active contacts
  size_t a_room;
  int nc_cap;
};

OST_HD size_t align8(size_t x) { return (x + 7) & ~size_t(7); }

// Storage split of one world's workspace.  SPLIT_LDS keeps everything in LDS;
// SPLIT_GLOBAL moves the m x m Schur matrix and the per-row Jacobian blocks
// (J, Y, G_lambda: 27 m doubles) to a per-workgroup slice of device memory,
// for worlds whose rows do not fit on chip.
enum { SPLIT_LDS = 0, SPLIT_GLOBAL = 1 };

// The Schur matrix is followed by kPadA spare doubles, so that the factor may
// read whole rounds of eight entries past the end of a row.
constexpr int kPadA = 8;

// Row stride of an m-row Schur matrix in the workspace: m rounded up to an odd
// count of doubles.  The factor and the solves give each lane its own row, so
// with an even stride (m = 36 for a robot on four wheels) the lanes of a
// wavefront meet on a quarter of the LDS banks; an odd stride spreads them
// over all banks.
OST_HD int lda(int m) { return m | 1; }
// Doubles of the Schur matrix's storage for up to mr rows.
OST_HD size_t schur_doubles(int mr) { return (size_t)mr * lda(mr) + kPadA; }

// Restart length of the adjoint's Krylov solve and the doubles its workspace
// takes: kKry + 1 basis vectors and the iterate over the 6 nb velocities, the
// (kKry + 1) x kKry Hessenberg matrix, and four short vectors.
constexpr int kKry = 8;
OST_HD size_t kry_doubles(const Caps& c) {
  return (size_t)(kKry + 2) * 6 * c.nb + (size_t)(kKry + 1) * kKry + 4 * kKry + 2;
}

OST_HD size_t world_glob_doubles(const Caps& c, int split) {
  return split == SPLIT_GLOBAL ? schur_doubles(c.mr) + (size_t)27 * c.mr : 0;
}

// Bytes of LDS one world needs for the given capacities, team size and split;
// `adjoint` adds the Krylov workspace of the adjoint kernel.
OST_HD size_t world_lds_bytes(const Caps& c, int team, int split = SPLIT_LDS, bool adjoint = false) {
  size_t d = adjoint ? kry_doubles(c) : 0, i = 0;
  d += (size_t)c.nb * (3 + 7 + 9 + 9 + 9 + 1 + 3 + 6 * 7 + 7 + 6);
  d += (size_t)c.nc * 23;
  d += (size_t)c.mr * 8;
  if (split == SPLIT_LDS) d += (size_t)c.mr * 27 + schur_doubles(c.mr);
  d += c.mr;
  d += c.nsv;
  d += (size_t)team + 8;
  i += (size_t)c.nc * 4 + (size_t)c.mr * 6 + c.ns + c.nb + 16;
  size_t feat = (size_t)(c.nc + c.ns) * sizeof(Feature);
  return d * 8 + align8(i * 4) + align8(feat);
}

// Carve one world's workspace from LDS (and, with SPLIT_GLOBAL, from `glob`).
OST_HD WorldMem carve(char* base, const Caps& c, int team, int split = SPLIT_LDS, double* glob = nullptr,
                      bool adjoint = false) {
  WorldMem M;
  double* p = (double*)base;
  auto take = [&](size_t n) { double* r = p; p += n; return r; };
  double* g = glob;
  auto gtake = [&](size_t n) {
    if (split == SPLIT_LDS) return take(n);
    double* r = g; g += n; return r;
  };
  M.xm = take(3 * c.nb); M.qm = take(7 * c.nb); M.Rm = take(9 * c.nb); M.Iw = take(9 * c.nb);
  M.Iwi = take(9 * c.nb); M.mass = take(c.nb); M.inert = take(3 * c.nb); M.fext = take(6 * c.nb);
  M.um = take(6 * c.nb); M.u = take(6 * c.nb); M.du = take(6 * c.nb); M.rdyn = take(6 * c.nb);
  M.ubest = take(6 * c.nb); M.ut = take(6 * c.nb); M.gq = take(7 * c.nb); M.kg = take(6 * c.nb);
  M.c_n = take(3 * c.nc); M.c_t1 = take(3 * c.nc); M.c_t2 = take(3 * c.nc); M.c_noff = take(c.nc);
  M.c_la = take(3 * c.nc); M.c_lb = take(3 * c.nc); M.c_r = take(c.nc); M.c_mu = take(c.nc);
  M.c_sn = take(c.nc); M.c_sf = take(c.nc); M.c_ax = take(3 * c.nc);
  M.J = gtake(12 * c.mr); M.Y = gtake(12 * c.mr); M.Gl = gtake(3 * c.mr);
  M.D = take(c.mr); M.res = take(c.mr);
  M.lam = take(c.mr); M.dlam = take(c.mr); M.lamt = take(c.mr); M.lambest = take(c.mr); M.Abar = take(c.mr);
  M.rmax = take(c.mr);
  M.A = gtake(schur_doubles(c.mr)); M.rhs = take(c.mr); M.sv_in = take(c.nsv);
  M.red = take(team); M.dscal = take(8);
  M.kv = M.kx = M.kh = M.kcs = M.ksn = M.kgv = M.ky = nullptr;
  if (adjoint) {
    const size_t n = 6 * (size_t)c.nb;
    M.kv = take((kKry + 1) * n); M.kx = take(n); M.kh = take((size_t)(kKry + 1) * kKry);
    M.kcs = take(kKry); M.ksn = take(kKry); M.kgv = take(kKry + 1); M.ky = take(kKry + 1);
  }
  int* q = (int*)p;
  auto itake = [&](size_t n) { int* r = q; q += n; return r; };
  M.c_slot = itake(c.nc); M.c_kind = itake(c.nc); M.c_a = itake(c.nc); M.c_b = itake(c.nc);
  M.r_kind = itake(c.mr); M.r_a = itake(c.mr); M.r_b = itake(c.mr); M.r_idx = itake(c.mr);
  M.r_sub = itake(c.mr); M.r_g = itake(c.mr);
  M.s_act = itake(c.ns); M.b_first = itake(c.nb); M.iscal = itake(16);
  char* f = (char*)(((uintptr_t)q + 7) & ~uintptr_t(7));
  M.c_feat = (Feature*)f;
  M.s_feat = M.c_feat + c.nc;
  M.a_room = schur_doubles(c.mr);
  M.nc_cap = c.nc;
  return M;
}

// Per-world view of the packed batch.
struct WorldRef {
  int w, b0, nb, j0, nj, s0, ns, o0, l0, c0, cap, nsv, m, nc;
  HmapRef hm;  // the world's heightmap (n = 0: none)
  int bw;  // half band width of the Schur matrix (rows i, j couple only if |i - j| <= bw)
  int nctrl;
};

OST_HD WorldRef world_ref(const Batch& B, int w) {
  WorldRef R;
  R.w = w;
  R.b0 = B.body_off[w];
  R.nb = B.body_off[w + 1] - R.b0;
  R.j0 = B.joint_off[w];
  R.nj = B.joint_off[w + 1] - R.j0;
  R.s0 = B.slot_off[w];
  R.ns = B.slot_off[w + 1] - R.s0;
  R.o0 = B.obs_off[w];
  R.l0 = B.lam_off[w];
  R.c0 = B.ctrl_off[w];
  R.nctrl = B.ctrl_off[w + 1] - R.c0;
  R.cap = B.contact_cap[w];
  R.nsv = 0;
  for (int j = 0; j < R.nj; ++j) {
    int a = B.joint_act[R.j0 + j];
    if (a == 2 || a == 3 || a == 4) R.nsv++;
  }
  R.m = 0;
  R.nc = 0;
  R.bw = 0;
  int hi = B.world_hmap ? B.world_hmap[w] : -1;
  R.hm.n = 0;
  R.hm.h = nullptr;
  R.hm.sp = B.hmap_spacing;
  R.hm.ox = R.hm.oy = 0.0;
  if (hi >= 0 && B.hmap_n >= 2) {
    R.hm.n = B.hmap_n;
    R.hm.h = B.hmap_heights + (size_t)hi * B.hmap_n * B.hmap_n;
    R.hm.ox = B.hmap_origin[2 * hi];
    R.hm.oy = B.hmap_origin[2 * hi + 1];
  }
  return R;
}

// --------------------------------------------------------------------------
// Row evaluation.  All inputs that the adjoint differentiates are of type T.
// --------------------------------------------------------------------------
template <class T> struct GroupIn {
  v3<T> xa, xb;      // body positions at q-
  m3<T> Ra, Rb;      // rotations at q-
  const T* ua;       // velocity iterate of body a (6)
  const T* ub;       // velocity iterate of body b (6) or null
  const T* lg;       // multipliers of the group (1 or 3)
  Frame<T> fr;       // contact frame (contact groups)
  T target;          // servo velocity target
};

// Residual rows r (raw), Jacobian rows J (12 each) and the value of the row
// scale D of one group: a joint row, a servo row, or a contact (n, t1, t2).
// Angle of a revolute joint at the poses Ra, Rb: that of R_b perp1_a from
// R_a perp1_a about R_a axis_a (zero where the two frames coincide), as
// atan2(y, x) of y = (pa x pb) . axis, x = pa . pb.
template <class T>
OST_HD void joint_angle_yx(const m3<T>& Ra, const m3<T>& Rb, const double* fr, T& y, T& x) {
  const v3<T> pa = mul(Ra, ld3<T>(fr + 9)), pb = mul(Rb, ld3<T>(fr + 9)), ax = mul(Ra, ld3<T>(fr + 15));
  y = dot(cross(pa, pb), ax);
  x = dot(pa, pb);
}
// The angle itself (kept out of line: it is needed once per servo and step).
__host__ __device__ __attribute__((noinline)) inline double joint_angle(const m3<double>& Ra, const m3<double>& Rb,
                                                                        const double* fr) {
  double y, x;
  joint_angle_yx(Ra, Rb, fr, y, x);
  return ::atan2(y, x);
}
// Its derivative alone, from dual poses: d atan2(y, x) = (x dy - y dx) / (x^2 + y^2).
OST_HD double joint_angle_der(const m3<dual>& Ra, const m3<dual>& Rb, const double* fr) {
  dual y, x;
  joint_angle_yx(Ra, Rb, fr, y, x);
  return (x.v * y.d - y.v * x.d) / (x.v * x.v + y.v * y.v);
}

template <class T, bool kRim = true>
OST_HD void eval_group(const Batch& B, const Params& P, const WorldRef& R, int kind, int idx, int sub,
                       int has_b, double r_prox, T mu, double sn, double sf, int ckind,
                       const GroupIn<T>& in, T* r, T* J, double* D) {
  const double h = P.h;
  const v3<T> zero = mk(T(0.0), T(0.0), T(0.0));
  T zu[6] = {T(0.0), T(0.0), T(0.0), T(0.0), T(0.0), T(0.0)};
  BodyIt<T> Ba = body_it(in.xa, in.ua, h);
  BodyIt<T> Bb = body_it(in.xb, in.ub ? in.ub : zu, h);
  int n = kind == RK_CONTACT ? 3 : 1;
#pragma unroll
  for (int t = 0; t < 36; ++t) if (t < 12 * n) J[t] = T(0.0);
  if (kind == RK_ANCHOR || kind == RK_AXIS) {
    const double* fr = B.joint_frame + 18 * (R.j0 + idx);
    if (kind == RK_ANCHOR) {  // Eq. (3): e_i . (x_a + R_a anchor_a - x_b - R_b anchor_b), E = 0
      v3<T> e = mk(T(sub == 0 ? 1.0 : 0.0), T(sub == 1 ? 1.0 : 0.0), T(sub == 2 ? 1.0 : 0.0));
      v3<T> aa = mul(in.Ra, ld3<T>(fr));
      v3<T> ab = mul(in.Rb, ld3<T>(fr + 3));
      T ca = pos_term(Ba, aa, e, J);
      T cb = pos_term(Bb, ab, e, J + 6);
      for (int t = 6; t < 12; ++t) J[t] = -J[t];
      r[0] = ca - cb;
    } else {  // axis alignment: (R_a perp) . (R_b axis_b)
      v3<T> p = mul(in.Ra, ld3<T>(fr + (sub == 0 ? 9 : 12)));
      v3<T> q = mul(in.Rb, ld3<T>(fr + 6));
      v3<T> pa = cay(Ba.k, p), qb = cay(Bb.k, q);
      v3<T> ga = cay_grad(Ba.k, p, qb), gb = cay_grad(Bb.k, q, pa);
      J[3] = ga.x * 0.5; J[4] = ga.y * 0.5; J[5] = ga.z * 0.5;
      J[9] = gb.x * 0.5; J[10] = gb.y * 0.5; J[11] = gb.z * 0.5;
      r[0] = dot(pa, qb);
    }
    D[0] = 1.0 / h;
    return;
  }
  if (kind == RK_SERVO) {  // Eq. (8): velocity target (alpha = 1/k_p, b = -u_bar) or position target
    const double* fr = B.joint_frame + 18 * (R.j0 + idx);
    double kp = B.joint_kp[R.j0 + idx];
    v3<T> ax = mul(in.Ra, ld3<T>(fr + 15));
    J[3] = -ax.x; J[4] = -ax.y; J[5] = -ax.z;
    J[9] = ax.x; J[10] = ax.y; J[11] = ax.z;
    if (B.joint_act[R.j0 + idx] == 4) {  // alpha = 1/(k_d + h k_p), b = -alpha k_p target, target = theta* - theta(q-)
      const double al = 1.0 / (B.joint_kd[R.j0 + idx] + h * kp);
      r[0] = dot(ax, Bb.w - Ba.w) + in.lg[0] * al - in.target * (al * kp);
    } else {
      r[0] = dot(ax, Bb.w - Ba.w) + in.lg[0] / kp - in.target;
    }
    D[0] = 1.0;
    return;
  }
  // contact group: normal row (Eq. (4), eps-smoothed FB) and friction rows (Eq. (7))
  const Frame<T>& F = in.fr;
  // the proxy reaches `depth` below its centre along n; dsup points from its
  // contact point to its centre (a rim circle's contact point turns with body
  // a's axis at q+)
  T depth = T(r_prox);
  v3<T> dsup = F.n;
  v3<T> a1 = zero;
  if (kRim && F.disc) {
    a1 = cay(Ba.k, F.ax);
    depth = rim_depth(F.n, a1, r_prox, &dsup);
  }
  T gap;
  if (ckind == 2) {
    gap = pos_term(Ba, F.la, F.n, J) - pos_term(Bb, F.lb, F.n, J + 6) - r_prox;
    for (int t = 6; t < 12; ++t) J[t] = -J[t];
  } else {
    gap = pos_term(Ba, F.la, F.n, J) - F.noff - depth;
    if (kRim && F.disc && val(depth) > 0.0) {
      // depth = r sqrt(1 - (n . a)^2), a = Cay(k) ax: d(-depth)/dk = (r^2 (n . a) / depth) grad_k(n . a)
      const v3<T> g = cay_grad(Ba.k, F.ax, F.n) * (dot(F.n, a1) * (r_prox * r_prox) / depth);
      J[3] += g.x * 0.5; J[4] += g.y * 0.5; J[5] += g.z * 0.5;
    }
  }
  T Bq = sn * in.lg[0];
  T S = ssqrt(gap * gap + Bq * Bq + P.eps * P.eps);
  r[0] = gap + Bq - S;
  double pa = 1.0 - val(gap) / val(S);
  D[0] = 1.0 / (h * (pa > P.dg ? pa : P.dg));
  // tangential velocity of the material points at the contact point at q+
  v3<T> lev_a = cay(Ba.k, F.la) - dsup * r_prox;
  v3<T> pc = Ba.x + lev_a;
  v3<T> lev_b = has_b ? pc - Bb.x : zero;
  T vt[2];
  for (int s = 0; s < 2; ++s) {
    const v3<T>& t = s == 0 ? F.t1 : F.t2;
    T* Jr = J + 12 * (1 + s);
    v3<T> wa = cross(lev_a, t);
    Jr[0] = t.x; Jr[1] = t.y; Jr[2] = t.z;
    Jr[3] = wa.x; Jr[4] = wa.y; Jr[5] = wa.z;
    T v = dot(t, Ba.v) + dot(wa, Ba.w);
    if (has_b) {
      v3<T> wb = cross(lev_b, t);
      Jr[6] = -t.x; Jr[7] = -t.y; Jr[8] = -t.z;
      Jr[9] = -wb.x; Jr[10] = -wb.y; Jr[11] = -wb.z;
      v = v - dot(t, Bb.v) - dot(wb, Bb.w);
    }
    vt[s] = v;
    D[1 + s] = 1.0;
  }
  // compliance weight W = (sqrt(s^2 + beta^2) - beta) / (mu lambda_n), s the
  // eps-smoothed slip speed, beta = sigma_f (mu lambda_n - |lambda_f|_eps)
  const T& ln = in.lg[0];
  T s2 = vt[0] * vt[0] + vt[1] * vt[1] + P.eps * P.eps;
  T lf = ssqrt(in.lg[1] * in.lg[1] + in.lg[2] * in.lg[2] + P.eps * P.eps);
  T beta = sf * (mu * ln - lf);
  T Q = ssqrt(s2 + beta * beta);
  T den = tmax(ln * mu, T(P.dg));
  T W = val(beta) > 0.0 ? s2 / ((Q + beta) * den) : (Q - beta) / den;
  r[1] = vt[0] + W * in.lg[1];
  r[2] = vt[1] + W * in.lg[2];
}

// Generalized Jacobian of the scaled rows of a contact group (Newton matrix
// rows): G_u = D dr/du (3 x 12) and G_lambda = D dr/d(lambda_n, lambda_t1,
// lambda_t2) (3 x 3), in closed form.  J and D are the outputs of eval_group
// at the same point.
template <bool kRim = true>
OST_HD void contact_G(const Params& P, const GroupIn<double>& in, int has_b, double r_prox, double mu, double sn,
                      double sf, int ckind, const double* J, const double* D, double* Gu, double* Gl) {
  const double h = P.h;
  double zu[6] = {0, 0, 0, 0, 0, 0};
  BodyIt<double> Ba = body_it(in.xa, in.ua, h);
  BodyIt<double> Bb = body_it(in.xb, in.ub ? in.ub : zu, h);
  const Frame<double>& F = in.fr;
  double depth = r_prox;
  v3<double> dsup = F.n, a1{0.0, 0.0, 0.0};
  if (kRim && F.disc) {
    a1 = cay(Ba.k, F.ax);
    depth = rim_depth(F.n, a1, r_prox, &dsup);
  }
  // normal row: r_n = gap + B - S, S = sqrt(gap^2 + B^2 + eps^2), B = sigma_n lambda_n
  double gap = dot(F.n, Ba.x + cay(Ba.k, F.la));
  if (ckind == 2) gap -= dot(F.n, Bb.x + cay(Bb.k, F.lb));
  else gap -= F.noff;
  gap -= depth;  // r_prox but for a rim circle
  double Bq = sn * in.lg[0];
  double S = ::sqrt(gap * gap + Bq * Bq + P.eps * P.eps);
  double pa = 1.0 - gap / S, pb = 1.0 - Bq / S;
  double c = pa / (pa > P.dg ? pa : P.dg);
  for (int q = 0; q < 12; ++q) Gu[q] = c * J[q];
  Gl[0] = D[0] * sn * pb;
  Gl[1] = 0.0;
  Gl[2] = 0.0;
  // friction rows: r_f = v_t + W lambda_f
  v3<double> lev_a = cay(Ba.k, F.la) - dsup * r_prox;
  v3<double> pc = Ba.x + lev_a;
  v3<double> lev_b = has_b ? pc - Bb.x : v3<double>{0, 0, 0};
  double vt[2], dv[2][12];
  for (int s = 0; s < 2; ++s) {
    const v3<double>& t = s == 0 ? F.t1 : F.t2;
    const double* Jr = J + 12 * (1 + s);
    double v = 0.0;
    for (int q = 0; q < 6; ++q) v += Jr[q] * in.ua[q];
    if (has_b) for (int q = 0; q < 6; ++q) v += Jr[6 + q] * in.ub[q];
    vt[s] = v;
    // d v_t / du, including the dependence of the lever arms on the iterate
    v3<double> twa = cross(t, Ba.w);
    v3<double> gwa = cay_grad(Ba.k, F.la, twa) * (0.5 * h);
    v3<double> dva = t, dwa = cross(lev_a, t) + gwa;
    if (kRim && F.disc && depth > 0.0) {
      // the rim's contact point turns with the axis a = Cay(k) ax: with
      // d = t x w, al = n . a, be = d . a, si = sqrt(1 - al^2), the lever's
      // part -r dsup gives -r grad_k (d . dsup), d . dsup = (d . n - al be) / si
      const double al = dot(F.n, a1), be = dot(twa, a1), si = depth / r_prox;
      const v3<double> ga = cay_grad(Ba.k, F.ax, F.n), gb = cay_grad(Ba.k, F.ax, twa);
      const v3<double> gf = ga * ((al * dot(twa, F.n) - be) / (si * si * si)) - gb * (al / si);
      dwa = dwa - gf * (r_prox * 0.5 * h);
    }
    for (int q = 6; q < 12; ++q) dv[s][q] = 0.0;
    if (has_b) {
      v3<double> twb = cross(t, Bb.w);
      dva = dva - twb * h;
      dwa = dwa - cay_grad(Ba.k, F.la, twb) * (0.5 * h);
      v3<double> dvb = twb * h - t, dwb = -cross(lev_b, t);
      dv[s][6] = dvb.x; dv[s][7] = dvb.y; dv[s][8] = dvb.z;
      dv[s][9] = dwb.x; dv[s][10] = dwb.y; dv[s][11] = dwb.z;
    }
    dv[s][0] = dva.x; dv[s][1] = dva.y; dv[s][2] = dva.z;
    dv[s][3] = dwa.x; dv[s][4] = dwa.y; dv[s][5] = dwa.z;
  }
  const double ln = in.lg[0], l1 = in.lg[1], l2 = in.lg[2];
  double s2 = vt[0] * vt[0] + vt[1] * vt[1] + P.eps * P.eps;
  double lf = ::sqrt(l1 * l1 + l2 * l2 + P.eps * P.eps);
  double beta = sf * (mu * ln - lf);
  double Q = ::sqrt(s2 + beta * beta);
  bool den_act = ln * mu >= P.dg;
  double den = den_act ? ln * mu : P.dg;
  double W = beta > 0.0 ? s2 / ((Q + beta) * den) : (Q - beta) / den;
  double dW_ds2 = 0.5 / (Q * den);
  double dW_db = -W / Q;
  double dW_dln = dW_db * sf * mu + (den_act ? -W / den * mu : 0.0);
  double dW_dl1 = dW_db * (-sf * l1 / lf), dW_dl2 = dW_db * (-sf * l2 / lf);
  double lt[2] = {l1, l2};
  for (int s = 0; s < 2; ++s) {
    double* G = Gu + 12 * (1 + s);
    for (int q = 0; q < 12; ++q) {
      double dW = dW_ds2 * 2.0 * (vt[0] * dv[0][q] + vt[1] * dv[1][q]);
      G[q] = dv[s][q] + lt[s] * dW;
    }
    double* Gs = Gl + 3 * (1 + s);
    Gs[0] = lt[s] * dW_dln;
    Gs[1] = (s == 0 ? W : 0.0) + lt[s] * dW_dl1;
    Gs[2] = (s == 1 ? W : 0.0) + lt[s] * dW_dl2;
  }
}

// Body-level terms of r_dyn = M~ (u - u-) - h f_ext - h J^T lambda (Eq. (10)),
// without the constraint forces: mass, world inertia and f_ext at q-.
template <class T>
OST_HD void body_terms(const Params& P, double mass, const double* inert, const m3<T>& R, const T* um, const T* u,
                       const v3<T>& torque, T* out6) {
  const double h = P.h;
  for (int k = 0; k < 3; ++k) out6[k] = mass * (u[k] - um[k]) - h * (mass * P.g[k]);
  v3<T> wm = mk(um[3], um[4], um[5]);
  v3<T> dw = mk(u[3] - um[3], u[4] - um[4], u[5] - um[5]);
  auto Iw = [&](const v3<T>& v) {
    v3<T> l = mulT(R, v);
    l = mk(l.x * inert[0], l.y * inert[1], l.z * inert[2]);
    return mul(R, l);
  };
  v3<T> gyro = -cross(wm, Iw(wm));
  v3<T> a = Iw(dw);
  v3<T> f = gyro + torque;
  out6[3] = a.x - h * f.x;
  out6[4] = a.y - h * f.y;
  out6[5] = a.z - h * f.z;
}

}  // namespace ost
