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
};

struct Params {
  double h, g[3], tol, eps, dg, dreg, d0;
  int32_t kmax, kmin, ls_max, refine;
};

enum { RK_ANCHOR = 0, RK_AXIS = 1, RK_SERVO = 2, RK_CONTACT = 3 };
enum { ST_CONVERGED = 1, ST_BUDGET = 2, ST_NONFINITE = 4, ST_REGULARIZED = 8, ST_OVERFLOW = 16 };

// Contact frame decided at q-: which feature of the static box (clamp flags)
// and the tangent seed axis.  Fixed for the whole step.
struct Feature {
  int8_t flag[3];
  int8_t inside, in_axis, in_side, tan_e;
};

// Contact frame at q- (templated: the adjoint differentiates it w.r.t. q-).
template <class T> struct Frame {
  v3<T> n, t1, t2;
  T noff;       // static features: plane offset n . c0
  v3<T> la;     // world offset of the proxy centre from body a at q-
  v3<T> lb;     // body-face contacts: world offset of the contact point from body b at q-
};

// Frame of a slot at q-.  With `decide`, the feature choice is made (value
// arithmetic) and written to F; otherwise F is used as given.
template <class T>
OST_HD Frame<T> slot_frame(int kind, const double* sreal, const double* obs, const v3<T>& xa, const m3<T>& Ra,
                           const v3<T>& xb, const m3<T>& Rb, Feature& F, bool decide, double* gap_out) {
  Frame<T> C;
  C.la = mul(Ra, ld3<T>(sreal));
  v3<T> P = xa + C.la;
  double r = sreal[3];
  C.noff = T(0.0);
  C.lb = mk(T(0.0), T(0.0), T(0.0));
  T gap;
  if (kind == 0) {  // plane z = 0
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
