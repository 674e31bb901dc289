// Per-world model of the batched backward-Euler contact step (Ostrich,
// Sec. III): kinematics, contact frames, constraint rows and their residuals.
//
// Every function is templated on the scalar type.  With `dual` (a value and
// one tangent) the same closed-form code gives directional derivatives, which
// the Newton step uses for the generalized Jacobian of the constraint rows and
// the adjoint uses for the geometric-stiffness and pose pull-back terms.
//
// Conventions: per body q = (x, y, z, qx, qy, qz, qw), u = (v, w) with v the
// centre-of-mass velocity and w the angular velocity, both in the world frame.
// The rotation after the kinematic substitution of Eq. (1) is
//   R(q-, u) = Cay(h w / 2) R(q-),  Cay(k) a = a + 2/(1+|k|^2) (k x a + k x (k x a)),
// which is the rotation of the normalised quaternion q- + h G(q-) u.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#define OST_HD __host__ __device__ __forceinline__

namespace ost {

// ------------------------------------------------------------------ dual --
struct dual {
  double v, d;
  OST_HD dual() : v(0.0), d(0.0) {}
  OST_HD dual(double x) : v(x), d(0.0) {}
  OST_HD dual(double x, double t) : v(x), d(t) {}
};
OST_HD dual operator+(dual a, dual b) { return dual(a.v + b.v, a.d + b.d); }
OST_HD dual operator-(dual a, dual b) { return dual(a.v - b.v, a.d - b.d); }
OST_HD dual operator-(dual a) { return dual(-a.v, -a.d); }
OST_HD dual operator*(dual a, dual b) { return dual(a.v * b.v, a.d * b.v + a.v * b.d); }
OST_HD dual operator/(dual a, dual b) {
  double q = a.v / b.v;
  return dual(q, (a.d - q * b.d) / b.v);
}
OST_HD dual operator+(dual a, double s) { return dual(a.v + s, a.d); }
OST_HD dual operator+(double s, dual a) { return dual(a.v + s, a.d); }
OST_HD dual operator-(dual a, double s) { return dual(a.v - s, a.d); }
OST_HD dual operator-(double s, dual a) { return dual(s - a.v, -a.d); }
OST_HD dual operator*(dual a, double s) { return dual(a.v * s, a.d * s); }
OST_HD dual operator*(double s, dual a) { return dual(a.v * s, a.d * s); }
OST_HD dual operator/(dual a, double s) { return dual(a.v / s, a.d / s); }
OST_HD dual operator/(double s, dual a) {
  double q = s / a.v;
  return dual(q, -q * a.d / a.v);
}
OST_HD dual& operator+=(dual& a, dual b) { a = a + b; return a; }
OST_HD dual& operator-=(dual& a, dual b) { a = a - b; return a; }
OST_HD dual sqrt(dual a) {
  double s = ::sqrt(a.v);
  return dual(s, a.d / (2.0 * s));
}
OST_HD double val(double x) { return x; }
OST_HD double val(dual x) { return x.v; }
OST_HD double der(double) { return 0.0; }
OST_HD double der(dual x) { return x.d; }
template <class T> OST_HD T tmax(T a, T b) { return val(a) >= val(b) ? a : b; }
OST_HD double ssqrt(double x) { return ::sqrt(x); }
OST_HD dual ssqrt(dual x) { return sqrt(x); }

// --------------------------------------------------------------- vectors --
template <class T> struct v3 {
  T x, y, z;
};
template <class T> OST_HD v3<T> mk(T a, T b, T c) { return v3<T>{a, b, c}; }
template <class T> OST_HD v3<T> ld3(const double* p) { return v3<T>{T(p[0]), T(p[1]), T(p[2])}; }
template <class T> OST_HD v3<T> operator+(const v3<T>& a, const v3<T>& b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T> OST_HD v3<T> operator-(const v3<T>& a, const v3<T>& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T> OST_HD v3<T> operator-(const v3<T>& a) { return {-a.x, -a.y, -a.z}; }
template <class T, class S> OST_HD v3<T> operator*(const v3<T>& a, S s) { return {a.x * s, a.y * s, a.z * s}; }
template <class T> OST_HD T dot(const v3<T>& a, const v3<T>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> OST_HD v3<T> cross(const v3<T>& a, const v3<T>& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class T> OST_HD T& at(v3<T>& a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }
template <class T> OST_HD T at(const v3<T>& a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }

// 3x3 matrix, row major
template <class T> struct m3 {
  T a[9];
};
template <class T> OST_HD v3<T> mul(const m3<T>& M, const v3<T>& v) {
  return {M.a[0] * v.x + M.a[1] * v.y + M.a[2] * v.z, M.a[3] * v.x + M.a[4] * v.y + M.a[5] * v.z,
          M.a[6] * v.x + M.a[7] * v.y + M.a[8] * v.z};
}
template <class T> OST_HD v3<T> mulT(const m3<T>& M, const v3<T>& v) {
  return {M.a[0] * v.x + M.a[3] * v.y + M.a[6] * v.z, M.a[1] * v.x + M.a[4] * v.y + M.a[7] * v.z,
          M.a[2] * v.x + M.a[5] * v.y + M.a[8] * v.z};
}

// Rotation matrix of the normalised quaternion (x, y, z, w).
template <class T> OST_HD m3<T> quat_to_R(T qx, T qy, T qz, T qw) {
  T n = ssqrt(qx * qx + qy * qy + qz * qz + qw * qw);
  T x = qx / n, y = qy / n, z = qz / n, w = qw / n;
  m3<T> R;
  R.a[0] = 1.0 - 2.0 * (y * y + z * z);
  R.a[1] = 2.0 * (x * y - z * w);
  R.a[2] = 2.0 * (x * z + y * w);
  R.a[3] = 2.0 * (x * y + z * w);
  R.a[4] = 1.0 - 2.0 * (x * x + z * z);
  R.a[5] = 2.0 * (y * z - x * w);
  R.a[6] = 2.0 * (x * z - y * w);
  R.a[7] = 2.0 * (y * z + x * w);
  R.a[8] = 1.0 - 2.0 * (x * x + y * y);
  return R;
}

// Cayley rotation Cay(k) a.
template <class T> OST_HD v3<T> cay(const v3<T>& k, const v3<T>& a) {
  T s = 2.0 / (1.0 + dot(k, k));
  v3<T> ka = cross(k, a);
  return a + (ka + cross(k, ka)) * s;
}
// Gradient with respect to k of d . Cay(k) a (d, a fixed vectors).
// f = d.a + s g,  s = 2/(1+|k|^2),  g = (a x d).k + (d.k)(a.k) - (d.a)|k|^2.
template <class T> OST_HD v3<T> cay_grad(const v3<T>& k, const v3<T>& a, const v3<T>& d) {
  T kk = dot(k, k);
  T s = 2.0 / (1.0 + kk);
  v3<T> axd = cross(a, d);
  T dk = dot(d, k), ak = dot(a, k), da = dot(d, a);
  T g = dot(axd, k) + dk * ak - da * kk;
  v3<T> gg = axd + d * ak + a * dk - k * (2.0 * da);
  // grad s = -s^2 k
  return gg * s - k * (s * s * g);
}

// ------------------------------------------------------------- batch data --
struct Batch {
  int32_t n_worlds;
  const int32_t* body_off;
  const double* body_mass;
  const double* body_inertia;
  const int32_t* joint_off;
  const int32_t* joint_body;
  const double* joint_frame;
  const int32_t* joint_act;
  const double* joint_kp;
  const int32_t* ctrl_off;
  const int32_t* slot_off;
  const int32_t* slot_int;
  const double* slot_real;
  const int32_t* obs_off;
  const double* obs_box;
  const int32_t* lam_off;
  const int32_t* contact_cap;
  const int32_t* world_hmap;
  int32_t hmap_n;
  double hmap_spacing;
  const double* hmap_origin;
  const double* hmap_heights;
  const double* joint_kd;
};

struct Params {
  double h, g[3], tol, eps, dg, dreg, d0;
  double dreg_adj;  // regularisation of the factor the adjoint solves with (the tape's)
  int32_t kmax, kmin, ls_max, refine;
  int32_t truncate;  // adjoint: contact geometry held fixed in the q- pull-back
  int32_t lin;       // Newton step: 0 banded LU of the Schur matrix, 1 matrix-free Krylov solve
  int32_t lin_iters; // Krylov products per Newton step at most
};

enum { RK_ANCHOR = 0, RK_AXIS = 1, RK_SERVO = 2, RK_CONTACT = 3 };
enum { ST_CONVERGED = 1, ST_BUDGET = 2, ST_NONFINITE = 4, ST_REGULARIZED = 8, ST_OVERFLOW = 16,
       ST_ADJ_INEXACT = 32, ST_LOSS_BODY = 64 };

// Contact frame decided at q-: which feature of the static box (clamp flags)
// and the tangent seed axis.  Fixed for the whole step.
struct Feature {
  int8_t flag[3];
  int8_t inside, in_axis, in_side, tan_e;
  int32_t hkey;  // heightmap slots: feature key (6 * vertex + kind), -1 when no candidate
};

// Heightmap of a world: n x n vertices at spacing sp from (ox, oy); vertex
// (i, j) is at (ox + i sp, oy + j sp, h[i n + j]); cell (i, j) is split along
// its (i,j)-(i+1,j+1) diagonal into T0 = (v_ij, v_i+1,j, v_i+1,j+1) and
// T1 = (v_ij, v_i+1,j+1, v_i,j+1).
struct HmapRef {
  const double* h;
  int n;
  double sp, ox, oy;
};

// Local features of the triangle mesh, each owned by one vertex (i, j): the
// vertex (kind 0), the edges to (i+1, j) (1), (i, j+1) (2) and (i+1, j+1) (3),
// the faces T0 (4) and T1 (5) of cell (i, j); key = 6 (i n + j) + kind.  A
// feature is a candidate contact for the point P when P's closest point on the
// mesh near it lies on it and is a local minimum of the distance to the mesh:
// a face whose plane projection of P is interior; an edge whose projection is
// interior and which P lies beyond, in the plane of every triangle sharing the
// edge; a vertex from which every neighbouring vertex points away from P.
OST_HD v3<double> hm_vertex(const HmapRef& H, int i, int j) {
  return v3<double>{H.ox + i * H.sp, H.oy + j * H.sp, H.h[i * H.n + j]};
}

// P beyond edge (a, b) of triangle (a, b, c), in the triangle's plane.
OST_HD bool hm_beyond(const v3<double>& a, const v3<double>& b, const v3<double>& c, const v3<double>& p) {
  v3<double> N = cross(b - a, c - a);
  return dot(cross(b - a, p - a), N) < 0.0;
}

// Whether feature `key` is a candidate for P, and then its contact normal n
// (unit; from the feature to P for vertices and edges, the upward normal for
// faces), the plane offset noff = n . C of its closest point C, and the
// distance (|P - C|, or |n . (P - C)| for faces).
template <class T>
OST_HD bool hm_feature(const HmapRef& H, int key, const v3<T>& P, v3<T>& n, T& noff, double* dist) {
  const int kind = key % 6, vi = key / 6, i = vi / H.n, j = vi - i * H.n, N1 = H.n - 1;
  const v3<double> A = hm_vertex(H, i, j);
  const v3<double> p{val(P.x), val(P.y), val(P.z)};
  if (kind == 0) {
    const int di[6] = {1, -1, 0, 0, 1, -1}, dj[6] = {0, 0, 1, -1, 1, -1};
    for (int k = 0; k < 6; ++k) {
      int a = i + di[k], b = j + dj[k];
      if (a < 0 || b < 0 || a > N1 || b > N1) continue;
      if (!(dot(p - A, hm_vertex(H, a, b) - A) < 0.0)) return false;
    }
    v3<T> d = P - v3<T>{T(A.x), T(A.y), T(A.z)};
    T dn = ssqrt(dot(d, d));
    if (!(val(dn) > 1e-12)) return false;
    n = d * (1.0 / dn);
    noff = n.x * A.x + n.y * A.y + n.z * A.z;
    if (dist) *dist = val(dn);
    return true;
  }
  if (kind <= 3) {
    v3<double> Bv = kind == 1 ? hm_vertex(H, i + 1, j) : (kind == 2 ? hm_vertex(H, i, j + 1) : hm_vertex(H, i + 1, j + 1));
    v3<double> e = Bv - A;
    double tv = dot(p - A, e) / dot(e, e);
    if (!(tv > 0.0 && tv < 1.0)) return false;
    // third vertices of the triangles sharing the edge
    if (kind == 1) {
      if (j + 1 <= N1 && !hm_beyond(A, Bv, hm_vertex(H, i + 1, j + 1), p)) return false;
      if (j - 1 >= 0 && !hm_beyond(A, Bv, hm_vertex(H, i, j - 1), p)) return false;
    } else if (kind == 2) {
      if (i + 1 <= N1 && !hm_beyond(A, Bv, hm_vertex(H, i + 1, j + 1), p)) return false;
      if (i - 1 >= 0 && !hm_beyond(A, Bv, hm_vertex(H, i - 1, j), p)) return false;
    } else {
      if (!hm_beyond(A, Bv, hm_vertex(H, i + 1, j), p)) return false;
      if (!hm_beyond(A, Bv, hm_vertex(H, i, j + 1), p)) return false;
    }
    v3<T> pa = P - v3<T>{T(A.x), T(A.y), T(A.z)};
    T tt = (pa.x * e.x + pa.y * e.y + pa.z * e.z) * (1.0 / dot(e, e));
    v3<T> C = v3<T>{A.x + tt * e.x, A.y + tt * e.y, A.z + tt * e.z};
    v3<T> d = P - C;
    T dn = ssqrt(dot(d, d));
    if (!(val(dn) > 1e-12)) return false;
    n = d * (1.0 / dn);
    noff = dot(n, C);
    if (dist) *dist = val(dn);
    return true;
  }
  v3<double> V1, V2;
  if (kind == 4) { V1 = hm_vertex(H, i + 1, j); V2 = hm_vertex(H, i + 1, j + 1); }
  else { V1 = hm_vertex(H, i + 1, j + 1); V2 = hm_vertex(H, i, j + 1); }
  v3<double> N = cross(V1 - A, V2 - A);
  N = N * (1.0 / ::sqrt(dot(N, N)));
  // interior test of the projection of P onto the face (edge functions with the normal)
  const v3<double>* Vs[3] = {&A, &V1, &V2};
  for (int k = 0; k < 3; ++k) {
    const v3<double>& Va = *Vs[k];
    const v3<double>& Vb = *Vs[(k + 1) % 3];
    if (!(dot(cross(Vb - Va, p - Va), N) > 0.0)) return false;
  }
  n = v3<T>{T(N.x), T(N.y), T(N.z)};
  noff = T(dot(N, A));
  if (dist) *dist = fabs(dot(N, p - A));
  return true;
}

// Order of terrain candidates: distance quantised to 1e-9 m, then key.
OST_HD bool hm_before(long long d, int key, long long d2, int key2) { return d < d2 || (d == d2 && key < key2); }

// Insert (d, key) into the sorted best list (bd, bk) of at most 4 entries.
OST_HD void hm_insert(long long* bd, int* bk, int& nb, long long d, int key) {
  const int K = 4;
  int pos = nb;
  while (pos > 0 && hm_before(d, key, bd[pos - 1], bk[pos - 1])) --pos;
  if (pos >= K) return;
  int last = nb < K ? nb : K - 1;
  for (int q = last; q > pos; --q) { bd[q] = bd[q - 1]; bk[q] = bk[q - 1]; }
  bd[pos] = d;
  bk[pos] = key;
  if (nb < K) ++nb;
}

// The four nearest candidate features within radius rc of P among the cells
// part, part + nparts, ... (row-major) of P's search range, sorted; returns
// how many.  The best four of the union of the parts' lists are the best
// four of the whole range, whatever the split.
OST_HD int hm_best4(const HmapRef& H, const v3<double>& P, double rc, int part, int nparts, long long* bd, int* bk) {
  int nb = 0;
  if (H.n < 2) return 0;
  // vertex range covering the search disc (clamped in floating point, so that
  // non-finite or far-away points give an empty or bounded range)
  const double reach = rc + 2.0 * H.sp, top = H.n - 1;
  double fi0 = floor((P.x - reach - H.ox) / H.sp), fi1 = ceil((P.x + reach - H.ox) / H.sp);
  double fj0 = floor((P.y - reach - H.oy) / H.sp), fj1 = ceil((P.y + reach - H.oy) / H.sp);
  if (!(fi0 >= 0.0)) fi0 = 0.0;
  if (!(fj0 >= 0.0)) fj0 = 0.0;
  if (!(fi1 <= top)) fi1 = top;
  if (!(fj1 <= top)) fj1 = top;
  if (!(fi0 <= top) || !(fj0 <= top) || !(fi1 >= 0.0) || !(fj1 >= 0.0) || !(rc >= 0.0)) return 0;
  const int i0 = (int)fi0, i1 = (int)fi1, j0 = (int)fj0, j1 = (int)fj1;
  const int nj = j1 - j0 + 1, ncell = (i1 - i0 + 1) * nj;
  for (int c = part; c < ncell; c += nparts) {
    const int i = i0 + c / nj, j = j0 + c % nj;
    for (int kind = 0; kind < 6; ++kind) {
      if ((kind == 1 || kind == 3 || kind >= 4) && i + 1 >= H.n) continue;
      if ((kind == 2 || kind == 3 || kind >= 4) && j + 1 >= H.n) continue;
      int key = 6 * (i * H.n + j) + kind;
      v3<double> nn;
      double no, dd;
      if (!hm_feature<double>(H, key, P, nn, no, &dd) || !(dd <= rc)) continue;
      hm_insert(bd, bk, nb, (long long)floor(dd / 1e-9), key);
    }
  }
  return nb;
}

// The rank-th nearest candidate feature within radius rc of P, ordered by
// distance quantised to 1e-9 m and then by key; -1 if there are fewer.
OST_HD int hm_select(const HmapRef& H, const v3<double>& P, double rc, int rank) {
  long long bd[4];
  int bk[4];
  if (rank < 0 || rank >= 4) return -1;
  const int nb = hm_best4(H, P, rc, 0, 1, bd, bk);
  return rank < nb ? bk[rank] : -1;
}

// Contact frame at q- (templated: the adjoint differentiates it w.r.t. q-).
template <class T> struct Frame {
  v3<T> n, t1, t2;
  T noff;       // static features: plane offset n . c0
  v3<T> la;     // world offset of the proxy centre from body a at q-
  v3<T> lb;     // body-face contacts: world offset of the contact point from body b at q-
  int disc;     // the proxy is a rim circle (a cylindrical wheel's edge), not a sphere
  v3<T> ax;     // rim circle: its unit axis in the world at q-
};

// A frame of constants as one of dual numbers with zero tangents (every field).
OST_HD v3<dual> lift3(const v3<double>& a) { return v3<dual>{dual(a.x), dual(a.y), dual(a.z)}; }
OST_HD Frame<dual> lift_frame(const Frame<double>& f) {
  Frame<dual> g;
  g.n = lift3(f.n);
  g.t1 = lift3(f.t1);
  g.t2 = lift3(f.t2);
  g.noff = dual(f.noff);
  g.la = lift3(f.la);
  g.lb = lift3(f.lb);
  g.disc = f.disc;
  g.ax = lift3(f.ax);
  return g;
}

// Depth of a rim circle of radius r and unit axis a below its centre along the
// unit normal n: its points are c + r p with p a unit vector normal to a, and
// n . p is least at p = -d, d = (n - (n . a) a) / |n - (n . a) a|, which gives
// r sqrt(1 - (n . a)^2).  Writes d (the contact point is c - r d).  A circle
// facing n (1 - (n . a)^2 at most 1e-12) touches with its whole rim: depth 0,
// d = 0.
template <class T> OST_HD T rim_depth(const v3<T>& n, const v3<T>& a, double r, v3<T>* d) {
  const T na = dot(n, a);
  const T s2 = 1.0 - na * na;
  if (!(val(s2) > 1e-12)) {
    *d = mk(T(0.0), T(0.0), T(0.0));
    return T(0.0);
  }
  const T sn = ssqrt(s2);
  *d = (n - a * na) * (1.0 / sn);
  return sn * r;
}

// Frame of a slot at q-.  With `decide`, the feature choice is made (value
// arithmetic) and written to F; otherwise F is used as given.
// Heightmap slots (kind 3) take the rank-th nearest mesh feature within the
// search radius rc (decided at q-; rc is only used when deciding), or, keyed,
// the feature already in F.hkey.
template <class T>
OST_HD Frame<T> slot_frame(int kind, const double* sreal, const double* obs, const v3<T>& xa, const m3<T>& Ra,
                           const v3<T>& xb, const m3<T>& Rb, Feature& F, bool decide, double* gap_out,
                           const HmapRef* hm = nullptr, int rank = 0, double rc = 0.0, bool keyed = false) {
  Frame<T> C;
  C.la = mul(Ra, ld3<T>(sreal));
  v3<T> P = xa + C.la;
  double r = sreal[3];
  C.noff = T(0.0);
  C.lb = mk(T(0.0), T(0.0), T(0.0));
  C.disc = kind != 2 && (sreal[6] != 0.0 || sreal[7] != 0.0 || sreal[8] != 0.0);
  C.ax = C.disc ? mul(Ra, ld3<T>(sreal + 6)) : mk(T(0.0), T(0.0), T(0.0));
  T gap;
  if (kind == 3) {  // heightmap feature
    if (decide && !keyed) F.hkey = hm ? hm_select(*hm, v3<double>{val(P.x), val(P.y), val(P.z)}, rc, rank) : -1;
    bool ok = F.hkey >= 0 && hm_feature<T>(*hm, F.hkey, P, C.n, C.noff, nullptr);
    if (!ok) {  // no candidate: an inactive frame
      C.n = mk(T(0.0), T(0.0), T(1.0));
      C.noff = T(-1e30);
    }
    gap = ok ? dot(C.n, P) - C.noff - r : T(1e30);
  } else if (kind == 0) {  // plane z = 0
    C.n = mk(T(0.0), T(0.0), T(1.0));
    gap = P.z - r;
  } else if (kind == 1) {  // static axis-aligned box
    T cl[3];
    double dd = 0.0;
    for (int i = 0; i < 3; ++i) {
      double lo = obs[i] - obs[3 + i], hi = obs[i] + obs[3 + i];
      double pv = val(at(P, i));
      if (decide) F.flag[i] = pv < lo ? -1 : (pv > hi ? 1 : 0);
      cl[i] = F.flag[i] < 0 ? T(lo) : (F.flag[i] > 0 ? T(hi) : at(P, i));
      double dv = pv - val(cl[i]);
      dd += dv * dv;
    }
    if (decide) {
      F.inside = (F.flag[0] == 0 && F.flag[1] == 0 && F.flag[2] == 0) || ::sqrt(dd) <= 1e-12;
      if (F.inside) {
        double best = 1e300;
        for (int i = 0; i < 3; ++i) {
          double lo = obs[i] - obs[3 + i], hi = obs[i] + obs[3 + i], pv = val(at(P, i));
          if (pv - lo < best) { best = pv - lo; F.in_axis = i; F.in_side = -1; }
          if (hi - pv < best) { best = hi - pv; F.in_axis = i; F.in_side = 1; }
        }
      }
    }
    if (!F.inside) {
      v3<T> d = mk(P.x - cl[0], P.y - cl[1], P.z - cl[2]);
      T dn = ssqrt(dot(d, d));
      C.n = d * (1.0 / dn);
      C.noff = dot(C.n, mk(cl[0], cl[1], cl[2]));
    } else {
      int i = F.in_axis;
      C.n = mk(T(i == 0 ? F.in_side : 0), T(i == 1 ? F.in_side : 0), T(i == 2 ? F.in_side : 0));
      double face = F.in_side < 0 ? obs[i] - obs[3 + i] : obs[i] + obs[3 + i];
      C.noff = T(face * F.in_side);
    }
    gap = dot(C.n, P) - C.noff - r;
  } else {  // kind 2: +z face of body b at half-height sreal[5]
    C.n = mul(Rb, mk(T(0.0), T(0.0), T(1.0)));
    v3<T> f0 = xb + C.n * sreal[5];
    T h0 = dot(C.n, P - f0);
    C.lb = P - C.n * h0 - xb;
    gap = h0 - r;
  }
  // a rim circle reaches rim_depth below its centre along n, not r
  if (C.disc && val(gap) < 1e29) {
    v3<T> d;
    gap = gap + r - rim_depth(C.n, C.ax, r, &d);
  }
  if (decide) F.tan_e = fabs(val(C.n.x)) > 0.9 ? 1 : 0;
  v3<T> e = F.tan_e ? mk(T(0.0), T(1.0), T(0.0)) : mk(T(1.0), T(0.0), T(0.0));
  v3<T> t = cross(C.n, e);
  C.t1 = t * (1.0 / ssqrt(dot(t, t)));
  C.t2 = cross(C.n, C.t1);
  if (gap_out) *gap_out = val(gap);
  return C;
}

// Kinematic state of one body at an iterate u (Eq. (1) substitution).
template <class T> struct BodyIt {
  v3<T> x;   // x- + h v
  v3<T> k;   // h w / 2
  v3<T> v, w;
};
template <class T> OST_HD BodyIt<T> body_it(const v3<T>& xm, const T* u, double h) {
  BodyIt<T> B;
  B.v = mk(u[0], u[1], u[2]);
  B.w = mk(u[3], u[4], u[5]);
  B.x = xm + B.v * h;
  B.k = B.w * (0.5 * h);
  return B;
}

// Position-level constraint with a world direction d: d . (x + Cay(k) a) and
// its velocity Jacobian row (1/h) d/du = (d, 1/2 grad_k(d . Cay(k) a)).
template <class T> OST_HD T pos_term(const BodyIt<T>& B, const v3<T>& a, const v3<T>& d, T* J6) {
  v3<T> g = cay_grad(B.k, a, d);
  J6[0] = d.x; J6[1] = d.y; J6[2] = d.z;
  J6[3] = g.x * 0.5; J6[4] = g.y * 0.5; J6[5] = g.z * 0.5;
  return dot(d, B.x + cay(B.k, a));
}

}  // namespace ost
