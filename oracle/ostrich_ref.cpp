// CPU oracle for the batched backward-Euler contact step and its adjoint.
//
// TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
// baseline call it; the GPU library never does.  Plain, single-threaded FP64,
// written from the paper (Ostrich, Sec. III).  Every derivative is taken by
// forward-mode dual numbers straight from the residual's definition, so the
// oracle contains no hand-derived Jacobian: the Newton Jacobian of a position
// constraint is d c(q(u)) / du / h, the exact implicit-function Jacobian is
// dF/d(u, lambda), and the pull-back is dF/d(q-, u-, a).
//
// The terrain narrow phase searches every feature of the mesh (brute force);
// its pins are the flat heightmap, which must reproduce the plane z = h0, and
// hand-placed points over single features.  A cylindrical wheel touches with
// the two circles of its rims (Sec. IV-D), each reaching r sqrt(1 - (n . a)^2)
// below its centre along a contact normal n; its pins compare against a
// brute-force minimum over the rim's points.
//
// Every part has a pin of its own, from closed forms, brute force, central
// differences or the paper's worked example (tests/test_oracle_pins*.py), and
// planted mistakes in compiled copies of this file fail those pins; no part is
// left unpinned.
#include "ostrich_ref.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>
#include <cstdio>
#include <cstdlib>

namespace {

// ---------------------------------------------------------------- duals ----
template <class T>
struct Dual {
  T v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(double x) : v(x), d(0.0) {}
  Dual(const T& a, const T& b) : v(a), d(b) {}
};

inline double val(double x) { return x; }
template <class T> double val(const Dual<T>& x) { return val(x.v); }

template <class T> Dual<T> operator+(const Dual<T>& a, const Dual<T>& b) { return Dual<T>(a.v + b.v, a.d + b.d); }
template <class T> Dual<T> operator-(const Dual<T>& a, const Dual<T>& b) { return Dual<T>(a.v - b.v, a.d - b.d); }
template <class T> Dual<T> operator-(const Dual<T>& a) { return Dual<T>(-a.v, -a.d); }
template <class T> Dual<T> operator*(const Dual<T>& a, const Dual<T>& b) { return Dual<T>(a.v * b.v, a.d * b.v + a.v * b.d); }
template <class T> Dual<T> operator/(const Dual<T>& a, const Dual<T>& b) {
  T q = a.v / b.v;
  return Dual<T>(q, (a.d - q * b.d) / b.v);
}
template <class T> Dual<T> operator+(const Dual<T>& a, double s) { return Dual<T>(a.v + s, a.d); }
template <class T> Dual<T> operator+(double s, const Dual<T>& a) { return Dual<T>(a.v + s, a.d); }
template <class T> Dual<T> operator-(const Dual<T>& a, double s) { return Dual<T>(a.v - s, a.d); }
template <class T> Dual<T> operator-(double s, const Dual<T>& a) { return Dual<T>(s - a.v, -a.d); }
template <class T> Dual<T> operator*(const Dual<T>& a, double s) { return Dual<T>(a.v * s, a.d * s); }
template <class T> Dual<T> operator*(double s, const Dual<T>& a) { return Dual<T>(a.v * s, a.d * s); }
template <class T> Dual<T> operator/(const Dual<T>& a, double s) { return Dual<T>(a.v / s, a.d / s); }
template <class T> Dual<T> operator/(double s, const Dual<T>& a) {
  T q = s / a.v;
  return Dual<T>(q, -(q * a.d) / a.v);
}
template <class T, class U> Dual<T>& operator+=(Dual<T>& a, const U& b) { a = a + b; return a; }
template <class T, class U> Dual<T>& operator-=(Dual<T>& a, const U& b) { a = a - b; return a; }
template <class T> Dual<T> sqrt(const Dual<T>& a) {
  using std::sqrt;
  T s = sqrt(a.v);
  return Dual<T>(s, a.d / (2.0 * s));
}
using std::sqrt;
template <class T> Dual<T> cos(const Dual<T>& a) {
  using std::cos;
  using std::sin;
  return Dual<T>(cos(a.v), -(sin(a.v) * a.d));
}
template <class T> Dual<T> atan2(const Dual<T>& y, const Dual<T>& x) {
  using std::atan2;
  T r2 = x.v * x.v + y.v * y.v;
  return Dual<T>(atan2(y.v, x.v), (x.v * y.d - y.v * x.d) / r2);
}
using std::atan2;
using std::cos;

template <class T> Dual<T> lift(const T& a) { return Dual<T>(a, T(0.0)); }
template <class T> Dual<T> seed(const T& a) { return Dual<T>(a, T(1.0)); }
template <class T> T vmax(const T& a, const T& b) { return val(a) >= val(b) ? a : b; }

// ------------------------------------------------------------- vectors ----
template <class T> struct V3 { T x, y, z; };
template <class T> V3<T> operator+(const V3<T>& a, const V3<T>& b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T> V3<T> operator-(const V3<T>& a, const V3<T>& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T> V3<T> operator-(const V3<T>& a) { return {-a.x, -a.y, -a.z}; }
template <class T, class S> V3<T> operator*(const V3<T>& a, const S& s) { return {a.x * s, a.y * s, a.z * s}; }
template <class T> T dot(const V3<T>& a, const V3<T>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> V3<T> cross(const V3<T>& a, const V3<T>& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class T> T norm(const V3<T>& a) { return sqrt(dot(a, a)); }
template <class T> V3<T> cst3(const double* p) { return {T(p[0]), T(p[1]), T(p[2])}; }
template <class T> V3<T> cst3(double a, double b, double c) { return {T(a), T(b), T(c)}; }
template <class T> V3<Dual<T>> lift3(const V3<T>& a) { return {lift(a.x), lift(a.y), lift(a.z)}; }
// the value of a vector with every derivative part dropped
template <class T> V3<T> const3(const V3<T>& a) { return {T(val(a.x)), T(val(a.y)), T(val(a.z))}; }

template <class T> struct Q4 { T x, y, z, w; };
// Hamilton product, (x, y, z, w) storage.
template <class T> Q4<T> qmul(const Q4<T>& a, const Q4<T>& b) {
  return {a.w * b.x + b.w * a.x + (a.y * b.z - a.z * b.y),
          a.w * b.y + b.w * a.y + (a.z * b.x - a.x * b.z),
          a.w * b.z + b.w * a.z + (a.x * b.y - a.y * b.x),
          a.w * b.w - (a.x * b.x + a.y * b.y + a.z * b.z)};
}
template <class T> Q4<T> qnormalize(const Q4<T>& q) {
  T n = sqrt(q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w);
  return {q.x / n, q.y / n, q.z / n, q.w / n};
}
// Rotation of v by the unit quaternion q: v + 2w (qv x v) + 2 qv x (qv x v).
template <class T> V3<T> qrot(const Q4<T>& q, const V3<T>& v) {
  V3<T> qv{q.x, q.y, q.z};
  V3<T> t = cross(qv, v) * 2.0;
  return v + t * q.w + cross(qv, t);
}
template <class T> V3<T> qrot_inv(const Q4<T>& q, const V3<T>& v) {
  Q4<T> c{-q.x, -q.y, -q.z, q.w};
  return qrot(c, v);
}

// ---------------------------------------------------------- world data ----
constexpr double kFaceEps = 1e-12;

struct JointD {
  int a, b, act, ctrl;
  double anc_a[3], anc_b[3], axis_b[3], p1[3], p2[3], axis_a[3], kp, kd;
};
struct SlotD {
  int kind, a, b, feat;
  double loc[3], r, mu, face_h;
  double ax[3];  // rim circle: unit axis in body a's frame; zero for a sphere or point
  bool disc;
};
// Heightmap terrain: an n x n vertex grid, vertex (i, j) at (ox + i sp,
// oy + j sp, z[i n + j]); each grid cell is cut along the diagonal from
// (i, j) to (i+1, j+1).
struct HmapD {
  const double* z = nullptr;
  int n = 0;
  double sp = 0, ox = 0, oy = 0;
  V3<double> vert(int i, int j) const { return {ox + sp * i, oy + sp * j, z[i * n + j]}; }
};
// Model parameters as the evaluation's number type.  With dual numbers, the
// parameter named by the current seed (a body's mass, a slot's friction
// coefficient or a joint's servo gain) carries derivative 1, so that one
// evaluation gives the residual's derivative with respect to it (Eq. (17)
// with xi a parameter).  No seed is set outside the parameter pull-back.
enum { PS_NONE = 0, PS_MASS = 1, PS_MU = 2, PS_KP = 3 };
thread_local int g_seed_kind = PS_NONE, g_seed_idx = -1;
template <class T> T param(double v, int kind, int idx) {
  if constexpr (std::is_same<T, double>::value) {
    (void)kind;
    (void)idx;
    return v;
  } else {
    return T(v, kind == g_seed_kind && idx == g_seed_idx ? 1.0 : 0.0);
  }
}

struct WorldD {
  int nb = 0, nctrl = 0, nservo = 0, lam_len = 0, cap = 0;
  HmapD hm;
  const double* mass = nullptr;
  const double* inertia = nullptr;
  std::vector<JointD> joints;
  std::vector<SlotD> slots;
  const double* obs = nullptr;
  int no = 0;
};

WorldD load_world(const ostrich_ref_batch* B, int w) {
  WorldD W;
  int b0 = B->body_off[w];
  W.nb = B->body_off[w + 1] - b0;
  W.mass = B->body_mass + b0;
  W.inertia = B->body_inertia + 3 * b0;
  int c = 0;
  for (int j = B->joint_off[w]; j < B->joint_off[w + 1]; ++j) {
    JointD J;
    J.a = B->joint_body[2 * j];
    J.b = B->joint_body[2 * j + 1];
    const double* f = B->joint_frame + 18 * j;
    for (int k = 0; k < 3; ++k) {
      J.anc_a[k] = f[k];
      J.anc_b[k] = f[3 + k];
      J.axis_b[k] = f[6 + k];
      J.p1[k] = f[9 + k];
      J.p2[k] = f[12 + k];
      J.axis_a[k] = f[15 + k];
    }
    J.act = B->joint_act[j];
    J.kp = B->joint_kp[j];
    J.kd = B->joint_kd ? B->joint_kd[j] : 0.0;
    J.ctrl = J.act ? c++ : -1;
    if (J.act == 2 || J.act == 3 || J.act == 4) W.nservo++;
    W.joints.push_back(J);
  }
  W.nctrl = c;
  for (int s = B->slot_off[w]; s < B->slot_off[w + 1]; ++s) {
    SlotD S;
    S.kind = B->slot_int[4 * s];
    S.a = B->slot_int[4 * s + 1];
    S.b = B->slot_int[4 * s + 2];
    S.feat = B->slot_int[4 * s + 3];
    const double* r = B->slot_real + 9 * s;
    for (int k = 0; k < 3; ++k) S.loc[k] = r[k];
    S.r = r[3];
    S.mu = r[4];
    S.face_h = r[5];
    for (int k = 0; k < 3; ++k) S.ax[k] = r[6 + k];
    S.disc = r[6] != 0.0 || r[7] != 0.0 || r[8] != 0.0;
    W.slots.push_back(S);
  }
  if (B->world_hmap && B->world_hmap[w] >= 0 && B->hmap_n >= 2) {
    int k = B->world_hmap[w];
    W.hm.n = B->hmap_n;
    W.hm.sp = B->hmap_spacing;
    W.hm.z = B->hmap_heights + (size_t)k * B->hmap_n * B->hmap_n;
    W.hm.ox = B->hmap_origin[2 * k];
    W.hm.oy = B->hmap_origin[2 * k + 1];
  }
  W.obs = B->obs_box + 6 * B->obs_off[w];
  W.no = B->obs_off[w + 1] - B->obs_off[w];
  W.lam_len = B->lam_off[w + 1] - B->lam_off[w];
  W.cap = B->contact_cap[w];
  return W;
}

struct Prm {
  double h, g[3], tol, eps, dg, dreg, d0, dreg_adj;
  int kmax, kmin, sigma_mode, newton_mode, ls_max, truncate;
};
Prm load_params(const ostrich_ref_params* p) {
  Prm P;
  P.h = p->h;
  for (int k = 0; k < 3; ++k) P.g[k] = p->gravity[k];
  P.tol = p->tol;
  P.eps = p->eps;
  P.dg = p->delta_g;
  P.dreg = p->delta_reg;
  P.dreg_adj = p->delta_reg_adj;
  P.d0 = p->delta0;
  P.kmax = p->k_max;
  P.kmin = std::min(p->k_min, p->k_max);
  P.sigma_mode = p->sigma_mode;
  P.newton_mode = p->newton_mode;
  P.ls_max = p->ls_max;
  P.truncate = p->truncate;
  return P;
}

// ------------------------------------------------------ kinematics (1) ----
// Eq. (1): q+ = q- + h G(q-) u, with G = blockdiag(I3, E(q)/2) and
// E(q) w = (w, 0) (x) q; the rotation is read from the normalised quaternion.
template <class T>
void body_pose(const T* qm, const T* ub, double h, V3<T>& x, Q4<T>& qn) {
  x = {qm[0] + h * ub[0], qm[1] + h * ub[1], qm[2] + h * ub[2]};
  Q4<T> q0{qm[3], qm[4], qm[5], qm[6]};
  Q4<T> om{ub[3], ub[4], ub[5], T(0.0)};
  Q4<T> dq = qmul(om, q0);
  Q4<T> qr{q0.x + (0.5 * h) * dq.x, q0.y + (0.5 * h) * dq.y, q0.z + (0.5 * h) * dq.z,
           q0.w + (0.5 * h) * dq.w};
  qn = qnormalize(qr);
}
template <class T> void raw_q_next(const T* qm, const T* ub, double h, T* out) {
  Q4<T> q0{qm[3], qm[4], qm[5], qm[6]};
  Q4<T> om{ub[3], ub[4], ub[5], T(0.0)};
  Q4<T> dq = qmul(om, q0);
  for (int k = 0; k < 3; ++k) out[k] = qm[k] + h * ub[k];
  out[3] = q0.x + (0.5 * h) * dq.x;
  out[4] = q0.y + (0.5 * h) * dq.y;
  out[5] = q0.z + (0.5 * h) * dq.z;
  out[6] = q0.w + (0.5 * h) * dq.w;
}
template <class T> Q4<T> prev_rot(const T* qm) { return qnormalize(Q4<T>{qm[3], qm[4], qm[5], qm[6]}); }

// World inertia I_w v = R (I_body o (R^T v)) at q-.
template <class T> V3<T> inertia_apply(const Q4<T>& R, const double* I, const V3<T>& v, bool inverse) {
  V3<T> l = qrot_inv(R, v);
  if (inverse) l = {l.x / I[0], l.y / I[1], l.z / I[2]};
  else l = {l.x * I[0], l.y * I[1], l.z * I[2]};
  return qrot(R, l);
}

// ------------------------------------------------- contact front end -----
// Active set and contact frame are fixed from q- for the whole step; the
// active set evolves only between steps.
// Terrain contacts (slot kind 3).  The mesh's local features are its
// vertices, its edges (open segments) and its triangles (open faces).  A
// feature is a candidate contact for the point P if the point of the feature
// nearest to P is a local minimum of the distance from P to the mesh surface:
// for a triangle, P projects into its interior; for an edge, P projects into
// the open segment and, in the plane of each triangle on the edge, lies on the
// far side of the edge from that triangle; for a vertex, P makes an obtuse
// angle with every edge leaving the vertex.  Candidates farther than the
// search radius are dropped, and slot k of a proxy takes the k-th candidate
// ordered by distance (quantised to 1e-9 m) and then by key.  Every feature is
// named by the vertex (i, j) that owns it and a kind: 0 the vertex, 1 edge to
// (i+1, j), 2 edge to (i, j+1), 3 edge to (i+1, j+1), 4 triangle
// (i,j),(i+1,j),(i+1,j+1), 5 triangle (i,j),(i+1,j+1),(i,j+1);
// key = 6 (i n + j) + kind.
constexpr double kDistQuantum = 1e-9;

// Barycentric coordinates of the projection of p onto the plane of (a, b, c).
void barycentric(const V3<double>& a, const V3<double>& b, const V3<double>& c, const V3<double>& p,
                 double& ua, double& ub, double& uc) {
  V3<double> e0 = b - a, e1 = c - a, e2 = p - a;
  double d00 = dot(e0, e0), d01 = dot(e0, e1), d11 = dot(e1, e1), d20 = dot(e2, e0), d21 = dot(e2, e1);
  double den = d00 * d11 - d01 * d01;
  ub = (d11 * d20 - d01 * d21) / den;
  uc = (d00 * d21 - d01 * d20) / den;
  ua = 1.0 - ub - uc;
}

// Normal n and plane offset noff = n . C of feature `key` for the point P
// (C the feature's point nearest to P), or false if it is not a candidate.
template <class T>
bool terrain_feature(const HmapD& H, int key, const V3<T>& P, V3<T>& n, T& noff, double* dist) {
  const int kind = key % 6, i = (key / 6) / H.n, j = (key / 6) % H.n, last = H.n - 1;
  const V3<double> A = H.vert(i, j);
  const V3<double> p{val(P.x), val(P.y), val(P.z)};
  auto exists = [&](int a, int b) { return a >= 0 && b >= 0 && a <= last && b <= last; };
  if (kind == 0) {
    const int nbr[6][2] = {{1, 0}, {0, 1}, {1, 1}, {-1, 0}, {0, -1}, {-1, -1}};
    for (const auto& d : nbr)
      if (exists(i + d[0], j + d[1]) && dot(H.vert(i + d[0], j + d[1]) - A, p - A) >= 0.0) return false;
    V3<T> d = P - cst3<T>(A.x, A.y, A.z);
    T len = norm(d);
    if (val(len) <= 1e-12) return false;
    n = d * (1.0 / len);
    noff = dot(n, cst3<T>(A.x, A.y, A.z));
    if (dist) *dist = val(len);
    return true;
  }
  if (kind <= 3) {
    const int bi = kind == 2 ? i : i + 1, bj = kind == 1 ? j : j + 1;
    const V3<double> B = H.vert(bi, bj);
    // third vertices of the (one or two) triangles on this edge
    int third[2][2], nt = 0;
    if (kind == 1) {
      if (exists(i + 1, j + 1)) { third[nt][0] = i + 1; third[nt][1] = j + 1; ++nt; }
      if (exists(i, j - 1)) { third[nt][0] = i; third[nt][1] = j - 1; ++nt; }
    } else if (kind == 2) {
      if (exists(i + 1, j + 1)) { third[nt][0] = i + 1; third[nt][1] = j + 1; ++nt; }
      if (exists(i - 1, j)) { third[nt][0] = i - 1; third[nt][1] = j; ++nt; }
    } else {
      third[0][0] = i + 1; third[0][1] = j;
      third[1][0] = i; third[1][1] = j + 1;
      nt = 2;
    }
    for (int k = 0; k < nt; ++k) {
      double ua, ub, uc;
      barycentric(A, B, H.vert(third[k][0], third[k][1]), p, ua, ub, uc);
      if (!(uc < 0.0)) return false;   // P is not beyond the edge in this triangle
    }
    const V3<double> e = B - A;
    T s = dot(P - cst3<T>(A.x, A.y, A.z), cst3<T>(e.x, e.y, e.z)) / dot(e, e);
    if (!(val(s) > 0.0 && val(s) < 1.0)) return false;
    V3<T> C = cst3<T>(A.x, A.y, A.z) + cst3<T>(e.x, e.y, e.z) * s;
    V3<T> d = P - C;
    T len = norm(d);
    if (val(len) <= 1e-12) return false;
    n = d * (1.0 / len);
    noff = dot(n, C);
    if (dist) *dist = val(len);
    return true;
  }
  const V3<double> B = kind == 4 ? H.vert(i + 1, j) : H.vert(i + 1, j + 1);
  const V3<double> Cv = kind == 4 ? H.vert(i + 1, j + 1) : H.vert(i, j + 1);
  V3<double> N = cross(B - A, Cv - A);
  N = N * (1.0 / norm(N));
  double ua, ub, uc;
  barycentric(A, B, Cv, p, ua, ub, uc);
  if (!(ua > 0.0 && ub > 0.0 && uc > 0.0)) return false;
  n = cst3<T>(N.x, N.y, N.z);
  noff = T(dot(N, A));
  if (dist) *dist = std::fabs(dot(N, p - A));
  return true;
}

// Brute force over every feature of the mesh: the rank-th candidate within rc.
int terrain_select(const HmapD& H, const V3<double>& P, double rc, int rank) {
  struct Cand { long long qd; int key; };
  std::vector<Cand> cands;
  for (int i = 0; i < H.n; ++i)
    for (int j = 0; j < H.n; ++j)
      for (int kind = 0; kind < 6; ++kind) {
        bool need_i = kind == 1 || kind == 3 || kind >= 4, need_j = kind == 2 || kind == 3 || kind >= 4;
        if ((need_i && i + 1 >= H.n) || (need_j && j + 1 >= H.n)) continue;
        int key = 6 * (i * H.n + j) + kind;
        V3<double> n;
        double noff, d;
        if (!terrain_feature<double>(H, key, P, n, noff, &d) || d > rc) continue;
        cands.push_back({(long long)std::floor(d / kDistQuantum), key});
      }
  std::sort(cands.begin(), cands.end(),
            [](const Cand& a, const Cand& b) { return a.qd < b.qd || (a.qd == b.qd && a.key < b.key); });
  return rank >= 0 && rank < (int)cands.size() ? cands[rank].key : -1;
}

struct Feature {
  int slot;
  int tkey;      // terrain: feature key, -1 if the slot has no candidate
  int flags[3];  // box: -1 clamped low, +1 clamped high, 0 free
  int inside;    // box: 1 if the proxy centre is inside (or on) the box
  int in_axis, in_side;
  int tan_e;     // tangent seed axis: 0 = e_x, 1 = e_y
};
template <class T> struct Contact {
  int slot, kind, a, b;
  double r, mu;
  V3<double> loc;
  V3<T> n, t1, t2, lb;
  T noff;
  bool disc;       // the proxy is a rim circle of axis ax (body a's frame)
  V3<double> ax;
};

// Support of a rim circle (radius r, unit axis a in the world) in direction
// -n: the circle's points are c + r p for unit p perpendicular to a, and
// n . p is least for p = -(n - (n . a) a) / |n - (n . a) a|, so the circle
// reaches r sqrt(1 - (n . a)^2) below its centre along n.  Returns that depth
// and the unit direction d = (n - (n . a) a) / |...| (the support point is
// c - r d).  A circle facing n (1 - (n . a)^2 at most 1e-12) touches with its
// whole rim: depth 0 and d = 0 (the centre stands for the rim).
template <class S> S rim_depth(const V3<S>& n, const V3<S>& a, double r, V3<S>* d) {
  S na = dot(n, a);
  S s2 = 1.0 - na * na;
  if (!(val(s2) > 1e-12)) {
    if (d) *d = cst3<S>(0, 0, 0);
    return S(0.0);
  }
  S sn = sqrt(s2);
  if (d) *d = (n - a * na) * (1.0 / sn);
  return sn * r;
}

template <class T>
Contact<T> contact_frame(const WorldD& W, const T* qprev, Feature& F, bool decide, double* gap_out,
                         V3<double>* pc_out) {
  const SlotD& S = W.slots[F.slot];
  Contact<T> C;
  C.slot = F.slot;
  C.kind = S.kind;
  C.a = S.a;
  C.b = S.b;
  C.r = S.r;
  C.mu = S.mu;
  C.loc = {S.loc[0], S.loc[1], S.loc[2]};
  C.disc = S.disc;
  C.ax = {S.ax[0], S.ax[1], S.ax[2]};
  const T* qa = qprev + 7 * S.a;
  Q4<T> Ra = prev_rot(qa);
  V3<T> P = V3<T>{qa[0], qa[1], qa[2]} + qrot(Ra, cst3<T>(S.loc));
  T gap;
  C.noff = T(0.0);
  C.lb = cst3<T>(0, 0, 0);
  if (S.kind == 3) {  // terrain feature, chosen at q- (search radius given by the caller)
    bool ok = F.tkey >= 0 && terrain_feature<T>(W.hm, F.tkey, P, C.n, C.noff, nullptr);
    if (!ok) {
      C.n = cst3<T>(0, 0, 1);
      C.noff = T(-1e30);
      gap = T(1e30);
    } else {
      gap = dot(C.n, P) - C.noff - S.r;
    }
  } else if (S.kind == 0) {  // ground plane z = 0
    C.n = cst3<T>(0, 0, 1);
    gap = P.z - S.r;
  } else if (S.kind == 1) {  // static axis-aligned box
    const double* o = W.obs + 6 * S.feat;
    T Pc[3] = {P.x, P.y, P.z};
    T cl[3];
    if (decide) {
      for (int i = 0; i < 3; ++i) {
        double lo = o[i] - o[3 + i], hi = o[i] + o[3 + i], pv = val(Pc[i]);
        F.flags[i] = pv < lo ? -1 : (pv > hi ? 1 : 0);
      }
    }
    double dd = 0;
    for (int i = 0; i < 3; ++i) {
      double lo = o[i] - o[3 + i], hi = o[i] + o[3 + i];
      cl[i] = F.flags[i] < 0 ? T(lo) : (F.flags[i] > 0 ? T(hi) : Pc[i]);
      double dv = val(Pc[i]) - val(cl[i]);
      dd += dv * dv;
    }
    if (decide) {
      F.inside = (F.flags[0] == 0 && F.flags[1] == 0 && F.flags[2] == 0) || std::sqrt(dd) <= kFaceEps;
      if (F.inside) {
        double best = 1e300;
        for (int i = 0; i < 3; ++i) {
          double lo = o[i] - o[3 + i], hi = o[i] + o[3 + i], pv = val(Pc[i]);
          if (pv - lo < best) { best = pv - lo; F.in_axis = i; F.in_side = -1; }
          if (hi - pv < best) { best = hi - pv; F.in_axis = i; F.in_side = 1; }
        }
      }
    }
    if (!F.inside) {
      V3<T> d{Pc[0] - cl[0], Pc[1] - cl[1], Pc[2] - cl[2]};
      T dn = norm(d);
      C.n = d * (1.0 / dn);
      C.noff = dot(C.n, V3<T>{cl[0], cl[1], cl[2]});
    } else {
      double e[3] = {0, 0, 0};
      int i = F.in_axis;
      e[i] = F.in_side;
      C.n = cst3<T>(e);
      double face = F.in_side < 0 ? o[i] - o[3 + i] : o[i] + o[3 + i];
      C.noff = T(face * F.in_side);
    }
    gap = dot(C.n, P) - C.noff - S.r;
  } else {  // kind 2: top (+z) face of body b at half-height face_h
    const T* qb = qprev + 7 * S.b;
    Q4<T> Rb = prev_rot(qb);
    V3<T> xb{qb[0], qb[1], qb[2]};
    C.n = qrot(Rb, cst3<T>(0, 0, 1));
    V3<T> f0 = xb + qrot(Rb, cst3<T>(0, 0, S.face_h));
    T h0 = dot(C.n, P - f0);
    V3<T> pc = P - C.n * h0;
    C.lb = qrot_inv(Rb, pc - xb);
    gap = h0 - S.r;
  }
  // a rim circle reaches r sqrt(1 - (n . a)^2) below its centre, not r
  V3<T> dsup = C.n;
  if (S.disc && S.kind != 2 && val(gap) < 1e29) gap = gap + S.r - rim_depth(C.n, qrot(Ra, cst3<T>(S.ax)), S.r, &dsup);
  if (decide) F.tan_e = std::fabs(val(C.n.x)) > 0.9 ? 1 : 0;
  V3<T> e = F.tan_e ? cst3<T>(0, 1, 0) : cst3<T>(1, 0, 0);
  V3<T> t = cross(C.n, e);
  C.t1 = t * (1.0 / norm(t));
  C.t2 = cross(C.n, C.t1);
  if (gap_out) *gap_out = val(gap);
  if (pc_out) {
    V3<T> pc = P - dsup * S.r;
    *pc_out = {val(pc.x), val(pc.y), val(pc.z)};
  }
  return C;
}

// Activation at q-: gap + h min(n . v_rel, 0) <= delta0 (the gap predicted
// after one step at the current approach speed), slots in ascending order, at
// most contact_cap of them.
void select_active(const WorldD& W, const Prm& P, const double* qm, const double* um,
                   std::vector<Feature>& act, bool& overflow) {
  act.clear();
  overflow = false;
  for (int s = 0; s < (int)W.slots.size(); ++s) {
    Feature F{};
    F.slot = s;
    F.tkey = -1;
    const SlotD& S = W.slots[s];
    if (S.kind == 3 && W.hm.n >= 2) {
      // search radius: proxy radius, activation margin and one step at the proxy centre's speed
      const double* q = qm + 7 * S.a;
      const double* ua = um + 6 * S.a;
      V3<double> arm = qrot(prev_rot(q), cst3<double>(S.loc));
      V3<double> vp = V3<double>{ua[0], ua[1], ua[2]} + cross(V3<double>{ua[3], ua[4], ua[5]}, arm);
      V3<double> pp{q[0] + arm.x, q[1] + arm.y, q[2] + arm.z};
      F.tkey = terrain_select(W.hm, pp, S.r + P.d0 + P.h * norm(vp), S.feat);
    }
    double gap;
    V3<double> pc;
    Contact<double> C = contact_frame<double>(W, qm, F, true, &gap, &pc);
    const double* ua = um + 6 * S.a;
    V3<double> xa{qm[7 * S.a], qm[7 * S.a + 1], qm[7 * S.a + 2]};
    V3<double> vr = V3<double>{ua[0], ua[1], ua[2]} + cross(V3<double>{ua[3], ua[4], ua[5]}, pc - xa);
    if (S.kind == 2) {
      const double* ub = um + 6 * S.b;
      V3<double> xb{qm[7 * S.b], qm[7 * S.b + 1], qm[7 * S.b + 2]};
      vr = vr - (V3<double>{ub[0], ub[1], ub[2]} + cross(V3<double>{ub[3], ub[4], ub[5]}, pc - xb));
    }
    // predicted gap after one step at the current approach speed
    double vn = dot(C.n, vr);
    if (gap + P.h * std::min(vn, 0.0) <= P.d0) {
      if ((int)act.size() < W.cap) act.push_back(F);
      else overflow = true;
    }
  }
}

// ------------------------------------------------------ residual (9)-(11) -
enum RowKind { R_ANCHOR = 0, R_AXIS = 1, R_SERVO = 2, R_NORMAL = 3, R_FRIC = 4 };

struct Layout {
  int nu, m, nj_rows, ns_rows;
  std::vector<int> kind, ra, rb, idx;  // idx: joint/servo/contact index
  std::vector<int> lam_slot;           // row -> lambda index in the slot-ordered state
};

Layout make_layout(const WorldD& W, const std::vector<Feature>& act) {
  Layout L;
  L.nu = 6 * W.nb;
  int nj = (int)W.joints.size();
  for (int j = 0; j < nj; ++j)
    for (int r = 0; r < 5; ++r) {
      L.kind.push_back(r < 3 ? R_ANCHOR : R_AXIS);
      L.ra.push_back(W.joints[j].a);
      L.rb.push_back(W.joints[j].b);
      L.idx.push_back(j);
      L.lam_slot.push_back(5 * j + r);
    }
  int sv = 0;
  for (int j = 0; j < nj; ++j)
    if (W.joints[j].act == 2 || W.joints[j].act == 3 || W.joints[j].act == 4) {
      L.kind.push_back(R_SERVO);
      L.ra.push_back(W.joints[j].a);
      L.rb.push_back(W.joints[j].b);
      L.idx.push_back(j);
      L.lam_slot.push_back(5 * nj + sv);
      ++sv;
    }
  int base = 5 * nj + W.nservo;
  for (int c = 0; c < (int)act.size(); ++c) {
    const SlotD& S = W.slots[act[c].slot];
    for (int r = 0; r < 3; ++r) {
      L.kind.push_back(r == 0 ? R_NORMAL : R_FRIC);
      L.ra.push_back(S.a);
      L.rb.push_back(S.kind == 2 ? S.b : -1);
      L.idx.push_back(c);
      L.lam_slot.push_back(base + 3 * act[c].slot + r);
    }
  }
  L.m = (int)L.kind.size();
  L.nj_rows = 5 * nj;
  L.ns_rows = W.nservo;
  return L;
}

template <class T> struct Eval {
  std::vector<T> F;        // raw residual [nu + m]: r_dyn, then constraint rows (Eqs. (9)-(11))
  std::vector<T> J;        // [m * 12] constraint Jacobian rows: body a (v, w), then body b (v, w)
  std::vector<double> D;   // [nu + m] row scale of the Newton system (1 on r_dyn)
  std::vector<double> Gu;  // [m * 12] d(D_i r_i)/d(u_a, u_b)          (constraint rows only)
  std::vector<double> Gl;  // [m * 3]  d(D_i r_i)/d(lambda of the row's group)
  std::vector<double> phia;// [m] FB derivative in the gap argument (normal rows)
  std::vector<double> Wf;  // [m] friction weight W of the contact (on its normal row)
  T norm2;
};

// Position-level constraint of a row as a function of the two poses.
template <class S>
S position_row(const WorldD& W, const Layout& L, int row, int sub, const Contact<S>& C,
               const V3<S>& xa, const Q4<S>& qa, const V3<S>& xb, const Q4<S>& qb) {
  int k = L.kind[row];
  if (k == R_ANCHOR) {
    const JointD& J = W.joints[L.idx[row]];
    V3<S> d = xa + qrot(qa, cst3<S>(J.anc_a)) - xb - qrot(qb, cst3<S>(J.anc_b));
    return sub == 0 ? d.x : (sub == 1 ? d.y : d.z);
  }
  if (k == R_AXIS) {
    const JointD& J = W.joints[L.idx[row]];
    V3<S> p = qrot(qa, cst3<S>(sub == 0 ? J.p1 : J.p2));
    return dot(p, qrot(qb, cst3<S>(J.axis_b)));
  }
  // normal contact: signed gap at q (first argument of the FB function, Eq. (4))
  V3<S> P = xa + qrot(qa, V3<S>{S(C.loc.x), S(C.loc.y), S(C.loc.z)});
  if (C.kind == 2) return dot(C.n, P - (xb + qrot(qb, C.lb))) - C.r;
  if (C.disc) return dot(C.n, P) - C.noff - rim_depth(C.n, qrot(qa, cst3<S>(C.ax.x, C.ax.y, C.ax.z)), C.r, (V3<S>*)nullptr);
  return dot(C.n, P) - C.noff - C.r;
}

template <class T> Contact<Dual<T>> lift_contact(const Contact<T>& C) {
  Contact<Dual<T>> D;
  D.slot = C.slot;
  D.kind = C.kind;
  D.a = C.a;
  D.b = C.b;
  D.r = C.r;
  D.mu = C.mu;
  D.loc = C.loc;
  D.n = lift3(C.n);
  D.t1 = lift3(C.t1);
  D.t2 = lift3(C.t2);
  D.lb = lift3(C.lb);
  D.noff = lift(C.noff);
  D.disc = C.disc;
  D.ax = C.ax;
  return D;
}

inline int group_size(const Layout& L, int g) { return L.kind[g] == R_NORMAL ? 3 : 1; }
inline int sub_index(const Layout& L, int row) {
  if (L.kind[row] == R_ANCHOR) return L.lam_slot[row] % 5;
  if (L.kind[row] == R_AXIS) return L.lam_slot[row] % 5 - 3;
  return 0;
}

// Velocity Jacobian rows of the two friction directions at the contact point
// at q (tangential relative velocity of the material points there), and the
// slip velocity v_t = J_f u.
template <class S>
void friction_rows(const Contact<S>& C, int b, const V3<S>& xa, const Q4<S>& qa, const V3<S>& xb,
                   const S* ua, const S* ub, S* Jf, S* vt) {
  // lever of the contact point: the proxy's support point in direction -n
  V3<S> dsup = C.n;
  if (C.disc) rim_depth(C.n, qrot(qa, cst3<S>(C.ax.x, C.ax.y, C.ax.z)), C.r, &dsup);
  V3<S> la = qrot(qa, V3<S>{S(C.loc.x), S(C.loc.y), S(C.loc.z)}) - dsup * C.r;
  V3<S> pc = xa + la;
  V3<S> lbv = b >= 0 ? pc - xb : cst3<S>(0, 0, 0);
  for (int r = 0; r < 2; ++r) {
    const V3<S>& t = r == 0 ? C.t1 : C.t2;
    S* Ji = Jf + 12 * r;
    V3<S> wa = cross(la, t);
    Ji[0] = t.x; Ji[1] = t.y; Ji[2] = t.z;
    Ji[3] = wa.x; Ji[4] = wa.y; Ji[5] = wa.z;
    for (int c = 6; c < 12; ++c) Ji[c] = S(0.0);
    if (b >= 0) {
      V3<S> wb = cross(lbv, t);
      Ji[6] = -t.x; Ji[7] = -t.y; Ji[8] = -t.z;
      Ji[9] = -wb.x; Ji[10] = -wb.y; Ji[11] = -wb.z;
    }
    S s(0.0);
    for (int c = 0; c < 6; ++c) s += Ji[c] * ua[c];
    if (b >= 0)
      for (int c = 0; c < 6; ++c) s += Ji[6 + c] * ub[c];
    vt[r] = s;
  }
}

// Raw residual rows of one row group (a joint row, a servo row, or the three
// rows of a contact) as a function of the group's local inputs.
template <class S>
void group_residual(const WorldD& W, const Prm& P, const Layout& L, int g, const Contact<S>* C, double sn,
                    double sf, const S* qa_m, const S* qb_m, const S* ua, const S* ub, const S* lg,
                    const S* ctrl, S* r, double* phia, double* wout = nullptr) {
  const double h = P.h;
  int k = L.kind[g], b = L.rb[g];
  V3<S> xa, xb = cst3<S>(0, 0, 0);
  Q4<S> qa, qb{S(0.0), S(0.0), S(0.0), S(1.0)};
  body_pose(qa_m, ua, h, xa, qa);
  if (b >= 0) body_pose(qb_m, ub, h, xb, qb);
  if (k == R_ANCHOR || k == R_AXIS) {  // Eq. (3) with E = 0
    Contact<S> dummy{};
    r[0] = position_row(W, L, g, sub_index(L, g), dummy, xa, qa, xb, qb);
    return;
  }
  if (k == R_SERVO) {  // Eq. (8), velocity target: J_c u + alpha lambda_c - u_bar, alpha = 1/k_p
    const JointD& J = W.joints[L.idx[g]];
    V3<S> ax = qrot(prev_rot(qa_m), cst3<S>(J.axis_a));
    S vel = ax.x * (ub[3] - ua[3]) + ax.y * (ub[4] - ua[4]) + ax.z * (ub[5] - ua[5]);
    // act 2: commanded joint speed; act 3: target 0 (axle damping beside a torque);
    // act 4: commanded joint angle, the implicit PD force k_p (theta* - theta+) -
    // k_d theta_dot+ with theta+ = theta(q-) + h theta_dot+, i.e. compliance
    // 1 / (k_d + h k_p) and b = k_p (theta(q-) - theta*) / (k_d + h k_p)
    const S kp = param<S>(J.kp, PS_KP, L.idx[g]);
    if (J.act == 4) {
      // joint angle at q-: of R_b p1 from R_a p1 about R_a axis_a
      Q4<S> ra = prev_rot(qa_m), rb = prev_rot(qb_m);
      V3<S> pa = qrot(ra, cst3<S>(J.p1)), pb = qrot(rb, cst3<S>(J.p1));
      V3<S> c = cross(pa, pb);
      S th = atan2(c.x * ax.x + c.y * ax.y + c.z * ax.z, pa.x * pb.x + pa.y * pb.y + pa.z * pb.z);
      S den = J.kd + h * kp;
      r[0] = vel + lg[0] / den + kp * (th - ctrl[J.ctrl]) / den;
    } else {
      r[0] = J.act == 2 ? vel + lg[0] / kp - ctrl[J.ctrl] : vel + lg[0] / kp;
    }
    return;
  }
  // normal row: eps-smoothed FB of (gap, sigma_n lambda_n), Eq. (4)
  S A = position_row(W, L, g, 0, *C, xa, qa, xb, qb);
  S B = sn * lg[0];
  S Sq = sqrt(A * A + B * B + P.eps * P.eps);
  r[0] = A + B - Sq;
  if (phia) *phia = 1.0 - val(A) / val(Sq);
  // friction rows, Eq. (7): r_f = J_f u + W lambda_f with the compliance weight
  // W = (sqrt(s^2 + beta^2) - beta) / (mu lambda_n) >= 0, s the eps-smoothed
  // slip speed and beta = sigma_f (mu lambda_n - |lambda_f|_eps).
  S Jf[24], vt[2];
  friction_rows(*C, b, xa, qa, xb, ua, ub, Jf, vt);
  const S& ln = lg[0];
  S s2 = vt[0] * vt[0] + vt[1] * vt[1] + P.eps * P.eps;
  S lf = sqrt(lg[1] * lg[1] + lg[2] * lg[2] + P.eps * P.eps);
  const S mu = param<S>(C->mu, PS_MU, C->slot);
  S beta = sf * (mu * ln - lf);
  S Q = sqrt(s2 + beta * beta);
  S den = vmax(mu * ln, S(P.dg));
  // (Q - beta) written as s^2 / (Q + beta) when beta > 0: same value, no cancellation
  S Wt = val(beta) > 0 ? s2 / ((Q + beta) * den) : (Q - beta) / den;
  r[1] = vt[0] + Wt * lg[1];
  r[2] = vt[1] + Wt * lg[2];
  if (wout) *wout = val(Wt);
}

// Constraint Jacobian rows J of one group.  A position-level row gets
// J = (1/h) d c(q(u)) / du (J at q+ with G at q-, Eqs. (1)-(2)), taken by
// forward-mode duals; velocity-level rows use their velocity Jacobian.
template <class T>
void group_jacobian(const WorldD& W, const Prm& P, const Layout& L, int g, const Contact<T>* C, const T* qa_m,
                    const T* qb_m, const T* ua, const T* ub, T* Jg) {
  typedef Dual<T> S;
  const double h = P.h;
  int k = L.kind[g], b = L.rb[g];
  int n = group_size(L, g);
  for (int t = 0; t < 12 * n; ++t) Jg[t] = T(0.0);
  if (k == R_SERVO) {
    const JointD& J = W.joints[L.idx[g]];
    V3<T> ax = qrot(prev_rot(qa_m), cst3<T>(J.axis_a));
    Jg[3] = -ax.x; Jg[4] = -ax.y; Jg[5] = -ax.z;
    Jg[9] = ax.x;  Jg[10] = ax.y; Jg[11] = ax.z;
    return;
  }
  Contact<S> Cs{};
  if (C) Cs = lift_contact(*C);
  S qa_s[7], qb_s[7];
  for (int t = 0; t < 7; ++t) {
    qa_s[t] = lift(qa_m[t]);
    qb_s[t] = b >= 0 ? lift(qb_m[t]) : S(0.0);
  }
  for (int side = 0; side < 2; ++side) {
    if (side == 1 && b < 0) continue;
    for (int c = 0; c < 6; ++c) {
      S us_a[6], us_b[6];
      for (int t = 0; t < 6; ++t) {
        us_a[t] = lift(ua[t]);
        us_b[t] = b >= 0 ? lift(ub[t]) : S(0.0);
      }
      if (side == 0) us_a[c] = seed(ua[c]);
      else us_b[c] = seed(ub[c]);
      V3<S> xa, xb = cst3<S>(0, 0, 0);
      Q4<S> qa, qb{S(0.0), S(0.0), S(0.0), S(1.0)};
      body_pose(qa_s, us_a, h, xa, qa);
      if (b >= 0) body_pose(qb_s, us_b, h, xb, qb);
      S gv = position_row(W, L, g, sub_index(L, g), Cs, xa, qa, xb, qb);
      Jg[6 * side + c] = gv.d / h;
    }
  }
  if (k == R_NORMAL) {
    V3<T> xa, xb = cst3<T>(0, 0, 0);
    Q4<T> qa, qb{T(0.0), T(0.0), T(0.0), T(1.0)};
    body_pose(qa_m, ua, h, xa, qa);
    if (b >= 0) body_pose(qb_m, ub, h, xb, qb);
    T vt[2];
    friction_rows(*C, b, xa, qa, xb, ua, ub, Jg + 12, vt);
  }
}

// Residual F(u, lambda; q-, u-, a) of Eqs. (9)-(11) with the kinematic
// substitution q = q- + h G(q-) u, its row scale, and (want_G, doubles only)
// the generalized Jacobian of the scaled constraint rows by forward duals.
template <class T>
void evaluate(const WorldD& W, const Prm& P, const Layout& L, const std::vector<Contact<T>>& C,
              const std::vector<double>& sig_n, const std::vector<double>& sig_f, const T* qm,
              const T* um, const T* ctrl, const T* u, const T* lam, Eval<T>& E, bool want_G = false) {
  const double h = P.h;
  const int nb = W.nb, m = L.m, nu = L.nu;
  E.F.assign(nu + m, T(0.0));
  E.J.assign(12 * m, T(0.0));
  E.D.assign(nu + m, 1.0);
  E.phia.assign(m, 0.0);
  E.Wf.assign(m, 0.0);
  if (want_G) {
    E.Gu.assign(12 * m, 0.0);
    E.Gl.assign(3 * m, 0.0);
  }
  std::vector<Q4<T>> Rm(nb);
  for (int b = 0; b < nb; ++b) Rm[b] = prev_rot(qm + 7 * b);
  // r_dyn = M~ (u - u-) - h (f_ext + J^T lambda)   (Eq. (10)); f_ext: gravity,
  // explicit gyroscopic term and actuator torques about the joint axis at q-.
  std::vector<V3<T>> tq(nb, cst3<T>(0, 0, 0));
  for (const JointD& J : W.joints)
    if (J.act == 1 || J.act == 3) {
      V3<T> ax = qrot(Rm[J.a], cst3<T>(J.axis_a));
      tq[J.b] = tq[J.b] + ax * ctrl[J.ctrl];
      tq[J.a] = tq[J.a] - ax * ctrl[J.ctrl];
    }
  for (int b = 0; b < nb; ++b) {
    const T mb = param<T>(W.mass[b], PS_MASS, b);
    for (int k = 0; k < 3; ++k) E.F[6 * b + k] = mb * (u[6 * b + k] - um[6 * b + k]) - h * (mb * P.g[k]);
    V3<T> wm{um[6 * b + 3], um[6 * b + 4], um[6 * b + 5]};
    V3<T> wk{u[6 * b + 3], u[6 * b + 4], u[6 * b + 5]};
    V3<T> gyro = -cross(wm, inertia_apply(Rm[b], W.inertia + 3 * b, wm, false));
    V3<T> Iw = inertia_apply(Rm[b], W.inertia + 3 * b, wk - wm, false);
    V3<T> fa = gyro + tq[b];
    E.F[6 * b + 3] = Iw.x - h * fa.x;
    E.F[6 * b + 4] = Iw.y - h * fa.y;
    E.F[6 * b + 5] = Iw.z - h * fa.z;
  }
  T zero6[6] = {T(0.0), T(0.0), T(0.0), T(0.0), T(0.0), T(0.0)};
  T zero7[7] = {T(0.0), T(0.0), T(0.0), T(0.0), T(0.0), T(0.0), T(1.0)};
  for (int g = 0; g < m; g += group_size(L, g)) {
    int k = L.kind[g], a = L.ra[g], b = L.rb[g], n = group_size(L, g);
    const Contact<T>* Cg = k == R_NORMAL ? &C[L.idx[g]] : nullptr;
    double sn = k == R_NORMAL ? sig_n[L.idx[g]] : 1.0, sf = k == R_NORMAL ? sig_f[L.idx[g]] : 1.0;
    const T* qa_m = qm + 7 * a;
    const T* qb_m = b >= 0 ? qm + 7 * b : zero7;
    // truncated pull-back (Sec. IV-D, terrain): a contact group sees its frame
    // and the bodies' poses at q- as constants, so no derivative with respect
    // to q- passes through it; values, and derivatives in u and lambda, are
    // those of the complete residual
    T qa_c[7], qb_c[7];
    Contact<T> Cc;
    if (P.truncate && k == R_NORMAL) {
      for (int t = 0; t < 7; ++t) { qa_c[t] = T(val(qa_m[t])); qb_c[t] = T(val(qb_m[t])); }
      Cc = *Cg;
      Cc.n = const3(Cg->n); Cc.t1 = const3(Cg->t1); Cc.t2 = const3(Cg->t2); Cc.lb = const3(Cg->lb);
      Cc.noff = T(val(Cg->noff));
      Cg = &Cc;
      qa_m = qa_c;
      qb_m = qb_c;
    }
    const T* ua = u + 6 * a;
    const T* ub = b >= 0 ? u + 6 * b : zero6;
    group_jacobian(W, P, L, g, Cg, qa_m, qb_m, ua, ub, &E.J[12 * g]);
    for (int r = 0; r < n; ++r) {
      const T* Ji = &E.J[12 * (g + r)];
      for (int c = 0; c < 6; ++c) E.F[6 * a + c] -= h * (Ji[c] * lam[g + r]);
      if (b >= 0)
        for (int c = 0; c < 6; ++c) E.F[6 * b + c] -= h * (Ji[6 + c] * lam[g + r]);
    }
    T rr[3];
    double pa = 0, wv = 0;
    group_residual(W, P, L, g, Cg, sn, sf, qa_m, qb_m, ua, ub, lam + g, ctrl, rr, &pa, &wv);
    E.Wf[g] = wv;
    for (int r = 0; r < n; ++r) E.F[nu + g + r] = rr[r];
    if (k == R_ANCHOR || k == R_AXIS) E.D[nu + g] = 1.0 / h;
    if (k == R_NORMAL) {
      E.phia[g] = pa;
      E.D[nu + g] = 1.0 / (h * std::max(pa, P.dg));
    }
    if constexpr (std::is_same<T, double>::value) {
      if (want_G) {
        typedef Dual<double> Dd;
        Contact<Dd> Cd{};
        if (Cg) Cd = lift_contact(*Cg);
        Dd qa_d[7], qb_d[7], ua_d[6], ub_d[6], lg_d[3], rd[3];
        std::vector<Dd> cd(std::max(W.nctrl, 1));
        for (int t = 0; t < W.nctrl; ++t) cd[t] = Dd(ctrl[t], 0.0);
        for (int t = 0; t < 7; ++t) { qa_d[t] = Dd(qa_m[t], 0.0); qb_d[t] = Dd(qb_m[t], 0.0); }
        for (int col = 0; col < 12 + n; ++col) {
          for (int t = 0; t < 6; ++t) {
            ua_d[t] = Dd(ua[t], col == t ? 1.0 : 0.0);
            ub_d[t] = Dd(ub[t], col == 6 + t ? 1.0 : 0.0);
          }
          for (int t = 0; t < n; ++t) lg_d[t] = Dd(lam[g + t], col == 12 + t ? 1.0 : 0.0);
          group_residual(W, P, L, g, Cg ? &Cd : nullptr, sn, sf, qa_d, qb_d, ua_d, ub_d, lg_d, cd.data(), rd,
                         nullptr);
          for (int r = 0; r < n; ++r) {
            double d = E.D[nu + g + r] * rd[r].d;
            if (col < 12) E.Gu[12 * (g + r) + col] = d;
            else E.Gl[3 * (g + r) + col - 12] = d;
          }
        }
      }
    }
  }
  T n2(0.0);
  for (int i = 0; i < nu + m; ++i) n2 += E.F[i] * E.F[i];
  E.norm2 = n2;
}

// ------------------------------------------------------- dense algebra ----
// M~^{-1} as a dense [nu x nu] matrix (block diagonal, Eq. (2)).
void mass_inverse(const WorldD& W, const double* qm, std::vector<double>& Mi) {
  int nu = 6 * W.nb;
  Mi.assign(nu * nu, 0.0);
  for (int b = 0; b < W.nb; ++b) {
    Q4<double> R = prev_rot(qm + 7 * b);
    for (int k = 0; k < 3; ++k) Mi[(6 * b + k) * nu + 6 * b + k] = 1.0 / W.mass[b];
    for (int c = 0; c < 3; ++c) {
      V3<double> e{c == 0 ? 1.0 : 0.0, c == 1 ? 1.0 : 0.0, c == 2 ? 1.0 : 0.0};
      V3<double> col = inertia_apply(R, W.inertia + 3 * b, e, true);
      Mi[(6 * b + 3) * nu + 6 * b + 3 + c] = col.x;
      Mi[(6 * b + 4) * nu + 6 * b + 3 + c] = col.y;
      Mi[(6 * b + 5) * nu + 6 * b + 3 + c] = col.z;
    }
  }
}

void dense_J(const Layout& L, const std::vector<double>& J12, std::vector<double>& Jd) {
  Jd.assign(L.m * L.nu, 0.0);
  for (int i = 0; i < L.m; ++i) {
    for (int c = 0; c < 6; ++c) Jd[i * L.nu + 6 * L.ra[i] + c] += J12[12 * i + c];
    if (L.rb[i] >= 0)
      for (int c = 0; c < 6; ++c) Jd[i * L.nu + 6 * L.rb[i] + c] += J12[12 * i + 6 + c];
  }
}

// Solve A x = b (A row-major n x n) by LU with partial pivoting.
bool lu_solve(std::vector<double> A, int n, std::vector<double>& b) {
  std::vector<int> piv(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[i * n + k]) > std::fabs(A[p * n + k])) p = i;
    if (A[p * n + k] == 0.0) return false;
    if (p != k) {
      for (int c = 0; c < n; ++c) std::swap(A[k * n + c], A[p * n + c]);
      std::swap(b[k], b[p]);
    }
    for (int i = k + 1; i < n; ++i) {
      double f = A[i * n + k] / A[k * n + k];
      A[i * n + k] = 0.0;
      for (int c = k + 1; c < n; ++c) A[i * n + c] -= f * A[k * n + c];
      b[i] -= f * b[k];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = b[i];
    for (int c = i + 1; c < n; ++c) s -= A[i * n + c] * b[c];
    b[i] = s / A[i * n + i];
  }
  return true;
}

// ------------------------------------------------------- per-world step ---
struct StepCtx {
  WorldD W;
  Prm P;
  std::vector<Feature> act;
  bool overflow = false;
  Layout L;
  std::vector<Contact<double>> C;
  std::vector<double> sig_n, sig_f, Mi;
  std::vector<double> qm, um, ctrl;
};

void prepare(StepCtx& X, const double* qm, const double* um, const double* ctrl) {
  int nb = X.W.nb;
  X.qm.assign(qm, qm + 7 * nb);
  X.um.assign(um, um + 6 * nb);
  X.ctrl.assign(X.W.nctrl + 1, 0.0);
  for (int t = 0; t < X.W.nctrl; ++t) X.ctrl[t] = ctrl[t];
  select_active(X.W, X.P, qm, um, X.act, X.overflow);
  X.L = make_layout(X.W, X.act);
  X.C.clear();
  for (Feature& F : X.act) X.C.push_back(contact_frame<double>(X.W, qm, F, false, nullptr, nullptr));
  mass_inverse(X.W, qm, X.Mi);
  // FB argument scaling from the Delassus diagonal J M~^-1 J^T at the warm start u = u-:
  // sigma_n = h^2 Abar_nn, sigma_f = h (Abar_t1t1 + Abar_t2t2) / 2.
  int nc = (int)X.act.size();
  X.sig_n.assign(nc, 1.0);
  X.sig_f.assign(nc, 1.0);
  if (X.P.sigma_mode) {
    Eval<double> E;
    std::vector<double> lam0(X.L.m, 0.0);
    evaluate<double>(X.W, X.P, X.L, X.C, X.sig_n, X.sig_f, qm, um, X.ctrl.data(), um, lam0.data(), E);
    std::vector<double> Jd;
    dense_J(X.L, E.J, Jd);
    int nu = X.L.nu;
    for (int i = 0; i < X.L.m; ++i) {
      if (X.L.kind[i] != R_NORMAL) continue;
      double ad[3];
      for (int r = 0; r < 3; ++r) {
        double s = 0;
        for (int p = 0; p < nu; ++p)
          for (int q = 0; q < nu; ++q) s += Jd[(i + r) * nu + p] * X.Mi[p * nu + q] * Jd[(i + r) * nu + q];
        ad[r] = s;
      }
      X.sig_n[X.L.idx[i]] = X.P.h * X.P.h * ad[0];
      X.sig_f[X.L.idx[i]] = X.P.h * 0.5 * (ad[1] + ad[2]);
    }
  }
}

// LU factorisation without pivoting (unit lower L and U in place).  A pivot is
// rejected when it is not finite or tiny against its row.
bool lu_nopivot(std::vector<double>& A, int n) {
  for (int k = 0; k < n; ++k) {
    double piv = A[k * n + k], rmax = 0.0;
    for (int j = k; j < n; ++j) rmax = std::max(rmax, std::fabs(A[k * n + j]));
    if (!std::isfinite(piv) || !(std::fabs(piv) > 1e-14 * rmax) || rmax == 0.0) return false;
    for (int i = k + 1; i < n; ++i) {
      double f = A[i * n + k] / piv;
      A[i * n + k] = f;
      for (int j = k + 1; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
    }
  }
  return true;
}
void lu_solve_np(const std::vector<double>& LU, int n, std::vector<double>& x) {
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < i; ++k) x[i] -= LU[i * n + k] * x[k];
  for (int i = n - 1; i >= 0; --i) {
    double s = x[i];
    for (int k = i + 1; k < n; ++k) s -= LU[i * n + k] * x[k];
    x[i] = s / LU[i * n + i];
  }
}

// Schur system of Eq. (12) at an iterate.  With the generalized Jacobian of the
// scaled constraint rows [G_u, G_lambda] and the dynamics block [M~, -h J^T]
// (geometric stiffness omitted):  A = G_u M~^-1 J^T + G_lambda / h
//                                      + dreg diag(J M~^-1 J^T),
// rhs = (G_u M~^-1 r_dyn - D r_con) / h.  newton_mode 1 freezes W and uses
// G_u = J, G_lambda = diag(C') as printed in the paper (symmetric A).
struct Schur {
  std::vector<double> Jd, Gud, Gld, Y, Abar, A, rhs, LU;
  double dreg_used = 0;
  bool regularized = false, ok = false;
};
void newton_rows(const StepCtx& X, const Eval<double>& E, int mode, std::vector<double>& Gud,
                 std::vector<double>& Gld) {
  const Layout& L = X.L;
  int m = L.m, nu = L.nu;
  Gud.assign(m * nu, 0.0);
  Gld.assign(m * m, 0.0);
  for (int g = 0; g < m; g += group_size(L, g)) {
    int n = group_size(L, g);
    for (int r = 0; r < n; ++r) {
      int i = g + r;
      bool lag = mode == 1 && L.kind[g] == R_NORMAL;
      for (int c = 0; c < 6; ++c) {
        double ga = lag ? E.J[12 * i + c] : E.Gu[12 * i + c];
        Gud[i * nu + 6 * L.ra[i] + c] += ga;
        if (L.rb[i] >= 0) Gud[i * nu + 6 * L.rb[i] + c] += lag ? E.J[12 * i + 6 + c] : E.Gu[12 * i + 6 + c];
      }
      for (int c = 0; c < n; ++c) Gld[i * m + g + c] = E.Gl[3 * i + c];
      if (lag && r > 0) {  // W frozen: d r_f / d lambda_f = W, no other coupling
        for (int c = 0; c < n; ++c) Gld[i * m + g + c] = 0.0;
        Gld[i * m + i] = E.Wf[g];
      }
    }
  }
}
void schur(const StepCtx& X, const Eval<double>& E, Schur& S, bool with_rhs, int mode, double dreg0 = -1.0) {
  int m = X.L.m, nu = X.L.nu;
  const double h = X.P.h;
  dense_J(X.L, E.J, S.Jd);
  newton_rows(X, E, mode, S.Gud, S.Gld);
  S.Y.assign(m * nu, 0.0);
  std::vector<double> YJ(m * nu, 0.0);
  for (int i = 0; i < m; ++i)
    for (int q = 0; q < nu; ++q) {
      double s = 0, t = 0;
      for (int p = 0; p < nu; ++p) {
        s += S.Gud[i * nu + p] * X.Mi[p * nu + q];
        t += S.Jd[i * nu + p] * X.Mi[p * nu + q];
      }
      S.Y[i * nu + q] = s;
      YJ[i * nu + q] = t;
    }
  S.Abar.assign(m * m, 0.0);
  std::vector<double> A0(m * m, 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      double s = 0, t = 0;
      for (int q = 0; q < nu; ++q) {
        s += S.Y[i * nu + q] * S.Jd[j * nu + q];
        t += YJ[i * nu + q] * S.Jd[j * nu + q];
      }
      A0[i * m + j] = s + S.Gld[i * m + j] / h;
      S.Abar[i * m + j] = t;
    }
  if (with_rhs) {
    S.rhs.assign(m, 0.0);
    for (int i = 0; i < m; ++i) {
      double s = 0;
      for (int q = 0; q < nu; ++q) s += S.Y[i * nu + q] * E.F[q];
      S.rhs[i] = (s - E.D[nu + i] * E.F[nu + i]) / h;
    }
  }
  double dreg = dreg0 >= 0.0 ? dreg0 : X.P.dreg;
  S.regularized = false;
  S.ok = false;
  for (int attempt = 0; attempt < 8; ++attempt) {
    S.A = A0;
    for (int i = 0; i < m; ++i) S.A[i * m + i] += dreg * S.Abar[i * m + i];
    S.LU = S.A;
    if (lu_nopivot(S.LU, m)) {
      S.ok = true;
      S.dreg_used = dreg;
      return;
    }
    S.regularized = true;
    dreg *= 10.0;
  }
}

// Friction safeguard: clamp |lambda_f| to mu lambda_n (Sec. III-B), with the
// same guard delta_g as the denominator of W so that a separated contact
// (lambda_n -> 0) keeps a reachable zero of its friction row.
void clamp_friction(const StepCtx& X, std::vector<double>& lam) {
  for (int i = 0; i < X.L.m; ++i) {
    if (X.L.kind[i] != R_NORMAL) continue;
    double mu = X.C[X.L.idx[i]].mu;
    double lim = std::max(mu * lam[i], X.P.dg);
    double n = std::sqrt(lam[i + 1] * lam[i + 1] + lam[i + 2] * lam[i + 2]);
    if (n > lim) {
      double s = n > 0 ? lim / n : 0.0;
      lam[i + 1] *= s;
      lam[i + 2] *= s;
    }
  }
}

struct StepResult {
  std::vector<double> u, lam;
  int status = 0, iters = 0;
  double resnorm = 0;
};

// Non-smooth Newton with best-iterate backtracking (Sec. III-C): a fixed
// budget, early exit at the tolerance, otherwise the iterate of smallest
// residual norm among k >= k_min (ties to the smaller k).
StepResult newton(StepCtx& X, const double* lam_prev_slots) {
  const Prm& P = X.P;
  int m = X.L.m, nu = X.L.nu;
  StepResult R;
  std::vector<double> u(X.um), lam(m, 0.0);
  for (int i = 0; i < m; ++i) lam[i] = lam_prev_slots[X.L.lam_slot[i]];
  clamp_friction(X, lam);
  Eval<double> E;
  evaluate<double>(X.W, P, X.L, X.C, X.sig_n, X.sig_f, X.qm.data(), X.um.data(), X.ctrl.data(), u.data(),
                   lam.data(), E, true);
  double nrm = std::sqrt(E.norm2);
  int status = X.overflow ? OSTRICH_REF_OVERFLOW : 0;
  std::vector<double> bu = u, bl = lam;
  double bn = nrm;
  bool have_best = P.kmin == 0;
  int iters = 0;
  if (!std::isfinite(nrm)) {
    R.u = u; R.lam = lam; R.status = status | OSTRICH_REF_NONFINITE | OSTRICH_REF_BUDGET; R.resnorm = nrm;
    return R;
  }
  if (nrm <= P.tol) {
    R.u = u; R.lam = lam; R.status = status | OSTRICH_REF_CONVERGED; R.resnorm = nrm;
    return R;
  }
  bool converged = false;
  for (int k = 1; k <= P.kmax; ++k) {
    Schur S;
    schur(X, E, S, true, P.newton_mode);
    if (S.regularized) status |= OSTRICH_REF_REGULARIZED;
    if (!S.ok) { status |= OSTRICH_REF_NONFINITE; break; }
    std::vector<double> dl = S.rhs;
    lu_solve_np(S.LU, m, dl);
    // Eq. (13): du = M~^{-1} (h J^T dlambda - r_dyn)
    std::vector<double> t(nu, 0.0), du(nu, 0.0);
    for (int q = 0; q < nu; ++q) {
      double s = -E.F[q];
      for (int i = 0; i < m; ++i) s += P.h * S.Jd[i * nu + q] * dl[i];
      t[q] = s;
    }
    for (int p = 0; p < nu; ++p) {
      double s = 0;
      for (int q = 0; q < nu; ++q) s += X.Mi[p * nu + q] * t[q];
      du[p] = s;
    }
    // Step length: alpha = 1, 1/2, ... (at most ls_max halvings) until the
    // residual norm decreases by the factor (1 - 1e-4 alpha); if none does,
    // the trial of smallest residual.  ls_max = 0 takes the full step.
    double alpha = 1.0, cur = nrm, best_t = 0.0;
    std::vector<double> ut(nu), lt(m), best_u, best_l;
    double best_n = INFINITY;
    Eval<double> Et, Ebest;
    for (int ls = 0; ls <= P.ls_max; ++ls) {
      for (int p = 0; p < nu; ++p) ut[p] = u[p] + alpha * du[p];
      for (int i = 0; i < m; ++i) lt[i] = lam[i] + alpha * dl[i];
      clamp_friction(X, lt);
      evaluate<double>(X.W, P, X.L, X.C, X.sig_n, X.sig_f, X.qm.data(), X.um.data(), X.ctrl.data(), ut.data(),
                       lt.data(), Et, true);
      double tn = std::sqrt(Et.norm2);
      bool ok = tn <= (1.0 - 1e-4 * alpha) * cur;
      if (tn < best_n || ok) {
        best_n = tn; best_u = ut; best_l = lt; Ebest = Et; best_t = alpha;
      }
      if (ok) break;
      alpha *= 0.5;
    }
    (void)best_t;
    u = best_u;
    lam = best_l;
    E = Ebest;
    nrm = std::sqrt(E.norm2);
    iters = k;
    if (std::getenv("OSTRICH_REF_TRACE")) {
      std::fprintf(stderr, "k=%d |F|=%.3e", k, nrm);
      if (std::getenv("OSTRICH_REF_TRACE")[0] == '2') {
        for (int i = 0; i < m; ++i) std::fprintf(stderr, " %.1e", E.F[nu + i]);
        std::fprintf(stderr, " | lam");
        for (int i = 0; i < m; ++i) std::fprintf(stderr, " %.2e", lam[i]);
        std::fprintf(stderr, " | dyn");
        for (int i = 0; i < nu; ++i) std::fprintf(stderr, " %.1e", E.F[i]);
      }
      std::fprintf(stderr, "\n");
    }
    if (!std::isfinite(nrm)) { status |= OSTRICH_REF_NONFINITE; break; }
    if (nrm <= P.tol) {
      bu = u; bl = lam; bn = nrm; converged = true; have_best = true;
      break;
    }
    if (k >= P.kmin && (!have_best || nrm < bn)) {
      bu = u; bl = lam; bn = nrm; have_best = true;
    }
  }
  R.u = bu;
  R.lam = bl;
  R.iters = iters;
  R.resnorm = bn;
  R.status = status | (converged ? OSTRICH_REF_CONVERGED : OSTRICH_REF_BUDGET);
  return R;
}

void finalize_q(const double* qm, const double* u, int nb, double h, double* qn) {
  for (int b = 0; b < nb; ++b) {
    double r[7];
    raw_q_next(qm + 7 * b, u + 6 * b, h, r);
    double n = std::sqrt(r[3] * r[3] + r[4] * r[4] + r[5] * r[5] + r[6] * r[6]);
    for (int k = 0; k < 3; ++k) qn[7 * b + k] = r[k];
    for (int k = 3; k < 7; ++k) qn[7 * b + k] = r[k] / n;
  }
}

// Exact Jacobian of the scaled residual at an iterate:
//   H = [[M~ - h d(J^T lambda)/du, -h J^T], [G_u, G_lambda + h dreg_adj diag(Abar)]],
// the multiplier block regularised by the adjoint's own delta_reg_adj (the
// root does not depend on the regularisation of the Newton iterations, but
// an adjoint solved with it would carry an O(delta_reg) bias).  Without
// `stiffness` the term - h d(J^T lambda)/du is left out: H is then the Newton
// matrix the forward iteration factors (the generalized Jacobian of the rows,
// the geometric stiffness of J^T lambda dropped), so an adjoint solved with it
// is the paper's reuse of the forward's matrix (Sec. III-D) for this forward.
void exact_jacobian(const StepCtx& X, const Eval<double>& E, const Schur& S, const double* u,
                    const double* lam, std::vector<double>& H, bool stiffness = true) {
  const Layout& L = X.L;
  const WorldD& W = X.W;
  const int nu = L.nu, m = L.m, n = nu + m;
  const double h = X.P.h;
  H.assign(n * n, 0.0);
  for (int p = 0; p < nu; ++p)
    for (int q = 0; q < nu; ++q) {
      int bp = p / 6, bq = q / 6;
      if (bp != bq) continue;
      int rp = p % 6, rq = q % 6;
      if (rp < 3 && rq < 3) H[p * n + q] = rp == rq ? W.mass[bp] : 0.0;
      else if (rp >= 3 && rq >= 3) {
        Q4<double> R = prev_rot(X.qm.data() + 7 * bp);
        V3<double> e{rq == 3 ? 1.0 : 0.0, rq == 4 ? 1.0 : 0.0, rq == 5 ? 1.0 : 0.0};
        V3<double> c = inertia_apply(R, W.inertia + 3 * bp, e, false);
        H[p * n + q] = rp == 3 ? c.x : (rp == 4 ? c.y : c.z);
      }
    }
  // geometric stiffness: - h d(J(u)^T lambda)/du, group by group with duals
  typedef Dual<double> Dd;
  Dd zero6[6], zero7[7];
  for (int t = 0; t < 6; ++t) zero6[t] = Dd(0.0);
  for (int t = 0; t < 7; ++t) zero7[t] = Dd(t == 6 ? 1.0 : 0.0);
  for (int g = 0; stiffness && g < m; g += group_size(L, g)) {
    int k = L.kind[g], a = L.ra[g], b = L.rb[g], ng = group_size(L, g);
    Contact<Dd> Cd{};
    if (k == R_NORMAL) Cd = lift_contact(X.C[L.idx[g]]);
    Dd qa[7], qb[7];
    for (int t = 0; t < 7; ++t) {
      qa[t] = Dd(X.qm[7 * a + t], 0.0);
      qb[t] = b >= 0 ? Dd(X.qm[7 * b + t], 0.0) : zero7[t];
    }
    for (int col = 0; col < (b >= 0 ? 12 : 6); ++col) {
      Dd ua[6], ub[6];
      for (int t = 0; t < 6; ++t) {
        ua[t] = Dd(u[6 * a + t], col == t ? 1.0 : 0.0);
        ub[t] = b >= 0 ? Dd(u[6 * b + t], col == 6 + t ? 1.0 : 0.0) : zero6[t];
      }
      Dd Jg[36];
      group_jacobian<Dd>(W, X.P, L, g, k == R_NORMAL ? &Cd : nullptr, qa, qb, ua, ub, Jg);
      int qcol = col < 6 ? 6 * a + col : 6 * b + col - 6;
      for (int r = 0; r < ng; ++r)
        for (int c = 0; c < 12; ++c) {
          if (c >= 6 && b < 0) continue;
          int prow = c < 6 ? 6 * a + c : 6 * b + c - 6;
          H[prow * n + qcol] -= h * Jg[12 * r + c].d * lam[g + r];
        }
    }
  }
  for (int i = 0; i < m; ++i)
    for (int q = 0; q < nu; ++q) {
      H[q * n + nu + i] = -h * S.Jd[i * nu + q];
      H[(nu + i) * n + q] = S.Gud[i * nu + q];
    }
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) H[(nu + i) * n + nu + j] = S.Gld[i * m + j];
  for (int i = 0; i < m; ++i) H[(nu + i) * n + nu + i] += h * X.P.dreg_adj * S.Abar[i * m + i];
}

// ------------------------------------------------------- adjoint ---------
// Gradients of L(s+) w.r.t. (q-, u-, a) through one step (Sec. III-D).
void adjoint_world(StepCtx& X, const double* u_star, const double* lam_slots, const double* gq_next,
                   const double* gu_next, double* gq_prev, double* gu_prev, double* g_ctrl, int mode,
                   double* g_mass = nullptr, double* g_mu = nullptr, double* g_kp = nullptr) {
  const Prm& P = X.P;
  const WorldD& W = X.W;
  const int nb = W.nb, nu = X.L.nu, m = X.L.m, n = nu + m;
  const double h = P.h;
  std::vector<double> lam(m);
  for (int i = 0; i < m; ++i) lam[i] = lam_slots[X.L.lam_slot[i]];
  Eval<double> E;
  evaluate<double>(W, P, X.L, X.C, X.sig_n, X.sig_f, X.qm.data(), X.um.data(), X.ctrl.data(), u_star,
                   lam.data(), E, true);
  Schur S;
  schur(X, E, S, false, mode == 1 ? 1 : P.newton_mode, P.dreg_adj);

  // loss cotangent on the raw (unnormalised) q+, and the total u-cotangent
  // b = g_u + h G(q-)^T g_q (the kinematic substitution transposed)
  std::vector<double> gqr(7 * nb);
  for (int b = 0; b < nb; ++b) {
    double r[7];
    raw_q_next(X.qm.data() + 7 * b, u_star + 6 * b, h, r);
    double nq = std::sqrt(r[3] * r[3] + r[4] * r[4] + r[5] * r[5] + r[6] * r[6]);
    double qh[4] = {r[3] / nq, r[4] / nq, r[5] / nq, r[6] / nq};
    const double* g = gq_next + 7 * b;
    double dotq = qh[0] * g[3] + qh[1] * g[4] + qh[2] * g[5] + qh[3] * g[6];
    for (int k = 0; k < 3; ++k) gqr[7 * b + k] = g[k];
    for (int k = 0; k < 4; ++k) gqr[7 * b + 3 + k] = (g[3 + k] - qh[k] * dotq) / nq;
  }
  std::vector<double> bvec(gu_next, gu_next + nu);
  std::vector<double> dq_prev(7 * nb, 0.0);
  for (int b = 0; b < nb; ++b) {
    for (int c = 0; c < 6; ++c) {  // d q_raw / d u (dual per velocity component)
      Dual<double> qs[7], us[6], out[7];
      for (int t = 0; t < 7; ++t) qs[t] = Dual<double>(X.qm[7 * b + t], 0.0);
      for (int t = 0; t < 6; ++t) us[t] = Dual<double>(u_star[6 * b + t], t == c ? 1.0 : 0.0);
      raw_q_next(qs, us, h, out);
      double s = 0;
      for (int t = 0; t < 7; ++t) s += out[t].d * gqr[7 * b + t];
      bvec[6 * b + c] += s;
    }
    for (int c = 0; c < 7; ++c) {  // d q_raw / d q-
      Dual<double> qs[7], us[6], out[7];
      for (int t = 0; t < 7; ++t) qs[t] = Dual<double>(X.qm[7 * b + t], t == c ? 1.0 : 0.0);
      for (int t = 0; t < 6; ++t) us[t] = Dual<double>(u_star[6 * b + t], 0.0);
      raw_q_next(qs, us, h, out);
      double s = 0;
      for (int t = 0; t < 7; ++t) s += out[t].d * gqr[7 * b + t];
      dq_prev[7 * b + c] = s;
    }
  }

  std::vector<double> w(n, 0.0);
  if (mode == 1) {
    // Paper mode, Eqs. (18)-(19), with the frozen-W Schur matrix A:
    // A w_lambda = -J M~^-1 b ;  w_u = -M~^-1 (b + J^T w_lambda)
    std::vector<double> wl(m);
    for (int i = 0; i < m; ++i) {
      double s = 0;
      for (int q = 0; q < nu; ++q) {
        double t = 0;
        for (int p = 0; p < nu; ++p) t += S.Jd[i * nu + p] * X.Mi[p * nu + q];
        s += t * bvec[q];
      }
      wl[i] = -s;
    }
    std::vector<double> At(m * m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) At[i * m + j] = S.A[j * m + i];
    lu_solve(At, m, wl);
    for (int p = 0; p < nu; ++p) {
      double s = 0;
      for (int q = 0; q < nu; ++q) {
        double t = bvec[q];
        for (int i = 0; i < m; ++i) t += S.Jd[i * nu + q] * wl[i];
        s += X.Mi[p * nu + q] * t;
      }
      w[p] = -s;
    }
    for (int i = 0; i < m; ++i) w[nu + i] = wl[i];
  } else {
    // Exact IFT, Eq. (16): H^T w = -[b; 0], H the full Jacobian of the scaled
    // residual (its multiplier block regularised by delta_reg_adj); mode 2
    // leaves out its geometric stiffness, solving with the forward's Newton
    // matrix instead.
    std::vector<double> H;
    exact_jacobian(X, E, S, u_star, lam.data(), H, mode != 2);
    std::vector<double> Ht(n * n);
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < n; ++c) Ht[r * n + c] = H[c * n + r];
    for (int i = 0; i < nu; ++i) w[i] = -bvec[i];
    lu_solve(Ht, n, w);
  }

  // Eq. (17): dL/dxi = w^T D dF/dxi (pull-back through the residual, contact
  // frames included), plus the direct kinematic term for q-.
  typedef Dual<double> Dd;
  auto pull = [&](int which, int comp) -> double {
    std::vector<Dd> qd(7 * nb), umd(6 * nb), cd(W.nctrl + 1), ud(nu), ld(m);
    for (int t = 0; t < 7 * nb; ++t) qd[t] = Dd(X.qm[t], which == 0 && t == comp ? 1.0 : 0.0);
    for (int t = 0; t < 6 * nb; ++t) umd[t] = Dd(X.um[t], which == 1 && t == comp ? 1.0 : 0.0);
    for (int t = 0; t <= W.nctrl; ++t) cd[t] = Dd(X.ctrl[t], which == 2 && t == comp ? 1.0 : 0.0);
    for (int t = 0; t < nu; ++t) ud[t] = Dd(u_star[t], 0.0);
    for (int t = 0; t < m; ++t) ld[t] = Dd(lam[t], 0.0);
    std::vector<Contact<Dd>> Cd;
    for (Feature F : X.act) Cd.push_back(contact_frame<Dd>(W, qd.data(), F, false, nullptr, nullptr));
    Eval<Dd> Ed;
    evaluate<Dd>(W, P, X.L, Cd, X.sig_n, X.sig_f, qd.data(), umd.data(), cd.data(), ud.data(), ld.data(), Ed);
    double s = 0;
    for (int r = 0; r < n; ++r) s += w[r] * E.D[r] * Ed.F[r].d;
    return s;
  };
  for (int t = 0; t < 7 * nb; ++t) gq_prev[t] = dq_prev[t] + pull(0, t);
  for (int t = 0; t < 6 * nb; ++t) gu_prev[t] = pull(1, t);
  for (int t = 0; t < W.nctrl; ++t) g_ctrl[t] = pull(2, t);
  // model parameters: the same pull-back with the parameter seeded instead
  auto pull_param = [&](int kind, int idx) -> double {
    g_seed_kind = kind;
    g_seed_idx = idx;
    const double s = pull(3, 0);
    g_seed_kind = PS_NONE;
    g_seed_idx = -1;
    return s;
  };
  if (g_mass)
    for (int t = 0; t < nb; ++t) g_mass[t] = pull_param(PS_MASS, t);
  if (g_mu)
    for (int t = 0; t < (int)W.slots.size(); ++t) g_mu[t] = pull_param(PS_MU, t);
  if (g_kp)
    for (int t = 0; t < (int)W.joints.size(); ++t) g_kp[t] = pull_param(PS_KP, t);
}

}  // namespace

// ================================================================ C ABI ====
extern "C" int ostrich_ref_step_forward(const ostrich_ref_batch* b, const ostrich_ref_params* p,
                                        const double* q_prev, const double* u_prev, const double* lam_prev,
                                        const double* ctrl, double* q_next, double* u_next, double* lam_next,
                                        int32_t* act_slot, int32_t* n_act, int32_t* status, int32_t* iters,
                                        double* resnorm) {
  if (!b || !p || !q_prev || !u_prev || !lam_prev || !q_next || !u_next || !lam_next) return -1;
  Prm P = load_params(p);
  for (int w = 0; w < b->n_worlds; ++w) {
    StepCtx X;
    X.W = load_world(b, w);
    X.P = P;
    for (const SlotD& s : X.W.slots) {
      if (s.kind == 3 && X.W.hm.n < 2) return -3;  // terrain slot without a heightmap
      if (s.disc && s.kind == 2) return -4;         // rim circles touch static features only
    }
    int b0 = b->body_off[w], c0 = b->ctrl_off[w], l0 = b->lam_off[w], s0 = b->slot_off[w];
    prepare(X, q_prev + 7 * b0, u_prev + 6 * b0, ctrl ? ctrl + c0 : nullptr);
    StepResult R = newton(X, lam_prev + l0);
    finalize_q(X.qm.data(), R.u.data(), X.W.nb, P.h, q_next + 7 * b0);
    for (int t = 0; t < 6 * X.W.nb; ++t) u_next[6 * b0 + t] = R.u[t];
    for (int t = 0; t < X.W.lam_len; ++t) lam_next[l0 + t] = 0.0;
    for (int i = 0; i < X.L.m; ++i) lam_next[l0 + X.L.lam_slot[i]] = R.lam[i];
    int ns = (int)X.W.slots.size();
    if (act_slot) {
      for (int s = 0; s < ns; ++s) act_slot[s0 + s] = -1;
      for (int c = 0; c < (int)X.act.size(); ++c) act_slot[s0 + c] = X.act[c].slot;
    }
    if (n_act) n_act[w] = (int)X.act.size();
    if (status) status[w] = R.status;
    if (iters) iters[w] = R.iters;
    if (resnorm) resnorm[w] = R.resnorm;
  }
  return 0;
}

extern "C" int ostrich_ref_step_adjoint(const ostrich_ref_batch* b, const ostrich_ref_params* p,
                                        const double* q_prev, const double* u_prev, const double* lam_prev,
                                        const double* ctrl, const double* u_next, const double* lam_next,
                                        const double* gq_next, const double* gu_next, double* gq_prev,
                                        double* gu_prev, double* g_ctrl, int32_t mode) {
  (void)lam_prev;
  if (!b || !p || !q_prev || !u_prev || !u_next || !lam_next || !gq_next || !gu_next) return -1;
  if (mode < 0 || mode > 2) return -1;
  Prm P = load_params(p);
  for (int w = 0; w < b->n_worlds; ++w) {
    StepCtx X;
    X.W = load_world(b, w);
    X.P = P;
    int b0 = b->body_off[w], c0 = b->ctrl_off[w], l0 = b->lam_off[w];
    prepare(X, q_prev + 7 * b0, u_prev + 6 * b0, ctrl ? ctrl + c0 : nullptr);
    std::vector<double> gc(X.W.nctrl + 1, 0.0);
    adjoint_world(X, u_next + 6 * b0, lam_next + l0, gq_next + 7 * b0, gu_next + 6 * b0, gq_prev + 7 * b0,
                  gu_prev + 6 * b0, gc.data(), mode);
    if (g_ctrl)
      for (int t = 0; t < X.W.nctrl; ++t) g_ctrl[c0 + t] = gc[t];
  }
  return 0;
}

extern "C" int ostrich_ref_step_adjoint_params(const ostrich_ref_batch* b, const ostrich_ref_params* p,
                                               const double* q_prev, const double* u_prev, const double* ctrl,
                                               const double* u_next, const double* lam_next, const double* gq_next,
                                               const double* gu_next, double* gq_prev, double* gu_prev,
                                               double* g_ctrl, double* g_mass, double* g_mu, double* g_kp,
                                               int32_t mode) {
  if (!b || !p || !q_prev || !u_prev || !u_next || !lam_next || !gq_next || !gu_next || !gq_prev || !gu_prev ||
      !g_mass || !g_mu || !g_kp || mode < 0 || mode > 2)
    return -1;
  Prm P = load_params(p);
  for (int w = 0; w < b->n_worlds; ++w) {
    StepCtx X;
    X.W = load_world(b, w);
    X.P = P;
    int b0 = b->body_off[w], c0 = b->ctrl_off[w], l0 = b->lam_off[w], s0 = b->slot_off[w], j0 = b->joint_off[w];
    prepare(X, q_prev + 7 * b0, u_prev + 6 * b0, ctrl ? ctrl + c0 : nullptr);
    std::vector<double> gc(X.W.nctrl + 1, 0.0);
    adjoint_world(X, u_next + 6 * b0, lam_next + l0, gq_next + 7 * b0, gu_next + 6 * b0, gq_prev + 7 * b0,
                  gu_prev + 6 * b0, gc.data(), mode, g_mass + b0, g_mu + s0, g_kp + j0);
    if (g_ctrl)
      for (int t = 0; t < X.W.nctrl; ++t) g_ctrl[c0 + t] = gc[t];
  }
  return 0;
}

extern "C" int ostrich_ref_spline_basis(int32_t T, int32_t K, double h, double* B) {
  if (T < 1 || K < 2 || !B) return -1;
  // natural cubic spline through K uniform knots on [0, T h]
  double dt = T * h / (K - 1);
  for (int j = 0; j < K; ++j) {
    std::vector<double> y(K, 0.0), Mv(K, 0.0);
    y[j] = 1.0;
    int ni = K - 2;
    if (ni > 0) {
      std::vector<double> A(ni * ni, 0.0), r(ni);
      for (int i = 0; i < ni; ++i) {
        A[i * ni + i] = 4.0 * dt;
        if (i > 0) A[i * ni + i - 1] = dt;
        if (i + 1 < ni) A[i * ni + i + 1] = dt;
        r[i] = 6.0 * (y[i + 2] - 2.0 * y[i + 1] + y[i]) / dt;
      }
      lu_solve(A, ni, r);
      for (int i = 0; i < ni; ++i) Mv[i + 1] = r[i];
    }
    for (int k = 0; k < T; ++k) {
      double t = k * h;
      int i = std::min((int)std::floor(t / dt), K - 2);
      double t0 = i * dt, t1 = (i + 1) * dt;
      double a = t1 - t, c = t - t0;
      B[k * K + j] = Mv[i] * a * a * a / (6 * dt) + Mv[i + 1] * c * c * c / (6 * dt) +
                     (y[i] - Mv[i] * dt * dt / 6) * a / dt + (y[i + 1] - Mv[i + 1] * dt * dt / 6) * c / dt;
    }
  }
  return 0;
}

// Terms of the shaped loss contributed by state k (1 <= k <= T): tracking and
// yaw alignment against the reference of step k and, at k = T, the final
// position, heading and velocity, for the loss body's pose q (7) and velocity
// u (6).  The yaw is the angle of the body x axis in the ground plane.
template <class S>
S state_loss(const ostrich_ref_loss& L, int W, int w, int k, int T, const S* q, const S* u) {
  V3<S> ex = qrot(prev_rot(q), cst3<S>(1.0, 0.0, 0.0));
  S psi = atan2(ex.y, ex.x);
  S s(0.0);
  if (L.w_track != 0.0 || L.w_yaw != 0.0) {
    const double* r = L.ref + 3 * ((size_t)(k - 1) * W + w);
    S dx = q[0] - r[0], dy = q[1] - r[1];
    s = s + (L.w_track / T) * (dx * dx + dy * dy);
    s = s + (L.w_yaw / T) * (1.0 - cos(psi - r[2]));
  }
  if (k == T) {
    const double* g = L.goal + 3 * w;
    S dx = q[0] - g[0], dy = q[1] - g[1];
    s = s + L.w_pos * (dx * dx + dy * dy);
    s = s + L.w_head * (1.0 - cos(psi - g[2]));
    s = s + L.w_vel * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  }
  return s;
}

// Cotangents of state_loss on the loss body's q (7) and u (6), by duals,
// added to gq and gu.
static void state_loss_grad(const ostrich_ref_loss& L, int W, int w, int k, int T, const double* q, const double* u,
                            double* gq, double* gu) {
  typedef Dual<double> Dd;
  for (int c = 0; c < 13; ++c) {
    Dd qd[7], ud[6];
    for (int t = 0; t < 7; ++t) qd[t] = Dd(q[t], c == t ? 1.0 : 0.0);
    for (int t = 0; t < 6; ++t) ud[t] = Dd(u[t], c == 7 + t ? 1.0 : 0.0);
    const double d = state_loss<Dd>(L, W, w, k, T, qd, ud).d;
    if (c < 7) gq[c] += d;
    else gu[c - 7] += d;
  }
}

// Rollout of every world with the final-xy loss (spec null) or the shaped loss.
static int rollout_impl(const ostrich_ref_batch* b, const ostrich_ref_params* p, const double* q0, const double* u0,
                        const double* knots, int32_t K, int32_t T, const int32_t* loss_body, const double* target,
                        const ostrich_ref_loss* spec, double* loss, double* qT, double* uT, double* g_q0,
                        double* g_u0, double* g_knots, int32_t mode, int32_t* status_or) {
  if (!b || !p || !q0 || !u0 || T < 1 || (!target && !spec)) return -1;
  Prm P = load_params(p);
  std::vector<double> B(T * std::max(K, 2), 0.0);
  if (K >= 2) ostrich_ref_spline_basis(T, K, P.h, B.data());
  const int NW = b->n_worlds;
  const bool per_step = spec && (spec->w_track != 0.0 || spec->w_yaw != 0.0);
  for (int w = 0; w < NW; ++w) {
    WorldD W = load_world(b, w);
    int b0 = b->body_off[w], c0 = b->ctrl_off[w];
    int nb = W.nb, nc = W.nctrl, nl = W.lam_len;
    std::vector<double> qs((T + 1) * 7 * nb), us((T + 1) * 6 * nb), ls((T + 1) * nl, 0.0), cs(T * (nc + 1), 0.0);
    std::copy(q0 + 7 * b0, q0 + 7 * b0 + 7 * nb, qs.begin());
    std::copy(u0 + 6 * b0, u0 + 6 * b0 + 6 * nb, us.begin());
    int st_or = 0;
    for (int k = 0; k < T; ++k) {
      for (int c = 0; c < nc; ++c) {
        double s = 0;
        for (int j = 0; j < K; ++j) s += B[k * K + j] * knots[(c0 + c) * K + j];
        cs[k * (nc + 1) + c] = s;
      }
      StepCtx X;
      X.W = W;
      X.P = P;
      prepare(X, &qs[k * 7 * nb], &us[k * 6 * nb], &cs[k * (nc + 1)]);
      StepResult R = newton(X, &ls[k * nl]);
      finalize_q(X.qm.data(), R.u.data(), nb, P.h, &qs[(k + 1) * 7 * nb]);
      std::copy(R.u.begin(), R.u.end(), us.begin() + (k + 1) * 6 * nb);
      for (int i = 0; i < X.L.m; ++i) ls[(k + 1) * nl + X.L.lam_slot[i]] = R.lam[i];
      st_or |= R.status;
    }
    if (status_or) status_or[w] = st_or;
    const int lb = loss_body[w];
    const double* qf = &qs[T * 7 * nb];
    auto q_at = [&](int k) { return &qs[k * 7 * nb + 7 * lb]; };
    auto u_at = [&](int k) { return &us[k * 6 * nb + 6 * lb]; };
    double dx = 0, dy = 0;
    if (!spec) {
      dx = qf[7 * lb] - target[2 * w];
      dy = qf[7 * lb + 1] - target[2 * w + 1];
      if (loss) loss[w] = dx * dx + dy * dy;
    } else if (loss) {
      double s = 0;
      for (int k = 1; k <= T; ++k)
        if (k == T || per_step) s += state_loss<double>(*spec, NW, w, k, T, q_at(k), u_at(k));
      double r = 0;
      for (int k = 0; k < T; ++k)
        for (int c = 0; c < nc; ++c) r += cs[k * (nc + 1) + c] * cs[k * (nc + 1) + c];
      loss[w] = s + spec->w_ctrl / T * r;
    }
    if (qT) std::copy(qf, qf + 7 * nb, qT + 7 * b0);
    if (uT) std::copy(&us[T * 6 * nb], &us[T * 6 * nb] + 6 * nb, uT + 6 * b0);
    if (!g_q0 && !g_u0 && !g_knots) continue;
    std::vector<double> gq(7 * nb, 0.0), gu(6 * nb, 0.0), gq2(7 * nb), gu2(6 * nb), gc(nc + 1);
    if (!spec) {
      gq[7 * lb] = 2 * dx;
      gq[7 * lb + 1] = 2 * dy;
    } else {
      state_loss_grad(*spec, NW, w, T, T, q_at(T), u_at(T), &gq[7 * lb], &gu[6 * lb]);
    }
    std::vector<double> gk(nc * std::max(K, 1), 0.0);
    for (int k = T - 1; k >= 0; --k) {
      StepCtx X;
      X.W = W;
      X.P = P;
      prepare(X, &qs[k * 7 * nb], &us[k * 6 * nb], &cs[k * (nc + 1)]);
      adjoint_world(X, &us[(k + 1) * 6 * nb], &ls[(k + 1) * nl], gq.data(), gu.data(), gq2.data(), gu2.data(),
                    gc.data(), mode);
      gq = gq2;
      gu = gu2;
      if (spec)  // control regulariser
        for (int c = 0; c < nc; ++c) gc[c] += 2.0 * spec->w_ctrl / T * cs[k * (nc + 1) + c];
      for (int c = 0; c < nc; ++c)
        for (int j = 0; j < K; ++j) gk[c * K + j] += B[k * K + j] * gc[c];
      if (per_step && k >= 1) state_loss_grad(*spec, NW, w, k, T, q_at(k), u_at(k), &gq[7 * lb], &gu[6 * lb]);
    }
    if (g_q0) std::copy(gq.begin(), gq.end(), g_q0 + 7 * b0);
    if (g_u0) std::copy(gu.begin(), gu.end(), g_u0 + 6 * b0);
    if (g_knots) std::copy(gk.begin(), gk.begin() + nc * K, g_knots + c0 * K);
  }
  return 0;
}

extern "C" int ostrich_ref_rollout(const ostrich_ref_batch* b, const ostrich_ref_params* p, const double* q0,
                                   const double* u0, const double* knots, int32_t K, int32_t T,
                                   const int32_t* loss_body, const double* target, double* loss, double* qT,
                                   double* uT, double* g_q0, double* g_u0, double* g_knots, int32_t mode,
                                   int32_t* status_or) {
  if (!target || mode < 0 || mode > 2) return -1;
  return rollout_impl(b, p, q0, u0, knots, K, T, loss_body, target, nullptr, loss, qT, uT, g_q0, g_u0, g_knots, mode,
                      status_or);
}

extern "C" int ostrich_ref_rollout_shaped(const ostrich_ref_batch* b, const ostrich_ref_params* p, const double* q0,
                                          const double* u0, const double* knots, int32_t K, int32_t T,
                                          const int32_t* loss_body, const ostrich_ref_loss* spec, double* loss,
                                          double* qT, double* uT, double* g_q0, double* g_u0, double* g_knots,
                                          int32_t mode, int32_t* status_or) {
  if (!spec || !spec->goal || ((spec->w_track != 0.0 || spec->w_yaw != 0.0) && !spec->ref) || mode < 0 || mode > 2)
    return -1;
  return rollout_impl(b, p, q0, u0, knots, K, T, loss_body, nullptr, spec, loss, qT, uT, g_q0, g_u0, g_knots, mode,
                      status_or);
}

extern "C" int ostrich_ref_inspect(const ostrich_ref_batch* b, const ostrich_ref_params* p, int32_t world,
                                   const double* q_prev, const double* u_prev, const double* ctrl,
                                   const double* u_it, const double* lam_it, int32_t* m_out, int32_t* nu_out,
                                   double* F, double* J, double* D, double* Gu, double* Gl, double* A, double* rhs,
                                   double* H, double* sigma, int32_t* act_slot) {
  if (!b || !p || world < 0 || world >= b->n_worlds) return -1;
  StepCtx X;
  X.W = load_world(b, world);
  X.P = load_params(p);
  int b0 = b->body_off[world], c0 = b->ctrl_off[world];
  prepare(X, q_prev + 7 * b0, u_prev + 6 * b0, ctrl ? ctrl + c0 : nullptr);
  int m = X.L.m, nu = X.L.nu, n = nu + m;
  if (m_out) *m_out = m;
  if (nu_out) *nu_out = nu;
  if (act_slot)
    for (int c = 0; c < (int)X.act.size(); ++c) act_slot[c] = X.act[c].slot;
  if (!u_it || !lam_it) return 0;
  Eval<double> E;
  evaluate<double>(X.W, X.P, X.L, X.C, X.sig_n, X.sig_f, X.qm.data(), X.um.data(), X.ctrl.data(), u_it, lam_it, E,
                   true);
  Schur S;
  schur(X, E, S, true, X.P.newton_mode);
  if (F) std::copy(E.F.begin(), E.F.end(), F);
  if (D) std::copy(E.D.begin(), E.D.end(), D);
  if (J) std::copy(S.Jd.begin(), S.Jd.end(), J);
  if (Gu) std::copy(S.Gud.begin(), S.Gud.end(), Gu);
  if (Gl) std::copy(S.Gld.begin(), S.Gld.end(), Gl);
  if (A) std::copy(S.A.begin(), S.A.end(), A);
  if (rhs) std::copy(S.rhs.begin(), S.rhs.end(), rhs);
  if (sigma)
    for (int i = 0; i < m; ++i) {
      int k = X.L.kind[i];
      if (k == R_NORMAL) sigma[i] = X.sig_n[X.L.idx[i]];
      else if (k == R_FRIC) sigma[i] = X.sig_f[X.L.idx[i]];
      else sigma[i] = 0.0;
    }
  if (H) {
    std::vector<double> Hs;
    exact_jacobian(X, E, S, u_it, lam_it, Hs);
    std::copy(Hs.begin(), Hs.begin() + n * n, H);
  }
  return 0;
}
