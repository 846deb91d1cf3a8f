// TEST INFRASTRUCTURE -- NOT PART OF THE PRODUCT PATH.
//
// Reference ("oracle") arithmetic for the CPU checker of the complex
// modified Gram-Schmidt least-squares solver.  Only tests/, the smoke check
// and the CPU-baseline leg of the benchmark may load the library built from
// this directory.  Nothing here is shared with the HIP kernels.
//
// Number formats (paper, Section 1: double double and quad double numbers
// are unevaluated sums of 2 resp. 4 hardware doubles; Dekker 1971 and
// Priest 1992 for their numerical properties):
//   dd = x0 + x1,            qd = x0 + x1 + x2 + x3.
//
// Formulations, written from the published mathematics, deliberately chosen
// to differ from the ones used on the GPU:
//   * TwoSum (Knuth / Moller), FastTwoSum (Dekker 1971), TwoProd with FMA.
//   * dd add: the "accurate double-word + double-word" sum and dd mul: the
//     FMA-based double-word product, both analysed by Joldes, Muller and
//     Popescu (ACM TOMS 2017).
//   * dd div: long division with three quotient digits; dd sqrt: one Newton
//     correction of the FP64 square root.
//   * qd: arbitrary-length expansion arithmetic (Shewchuk 1997, growing an
//     expansion with zero elimination).  Every sum and every product of
//     limbs is formed EXACTLY as an expansion, then rounded to four limbs by
//     successive extraction of the leading double.  qd div: long division
//     with five quotient digits against an exact remainder; qd sqrt: Newton
//     iteration with an exact residual.
// Compile with -ffp-contract=off and without fast-math: every operation
// below relies on IEEE round-to-nearest of each individual + - * and fma.
#pragma once
#include <cmath>
#include <cstring>

namespace orc {

// ----------------------------------------------------------------- EFTs ----
static inline void two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
static inline void fast_two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  e = b - (s - a);
}
static inline void two_prod(double a, double b, double &p, double &e) {
  p = a * b;
  e = std::fma(a, b, -p);
}

// --------------------------------------------------------------- double ----
static inline double add(double a, double b) { return a + b; }
static inline double sub(double a, double b) { return a - b; }
static inline double mul(double a, double b) { return a * b; }
static inline double div_(double a, double b) { return a / b; }
static inline double sqrt_(double a) { return std::sqrt(a); }
static inline double neg(double a) { return -a; }
static inline bool is_zero(double a) { return a == 0.0; }
static inline bool is_finite(double a) { return std::isfinite(a); }
static inline double hi(double a) { return a; }

// ------------------------------------------------------------------- dd ----
struct DD {
  double x[2];
};
static inline DD dd_make(double h, double l) { DD r; r.x[0] = h; r.x[1] = l; return r; }

// Accurate double-word + double-word (Joldes-Muller-Popescu 2017, Alg. 6);
// relative error below 3u^2 + 13u^3, u = 2^-53.
static inline DD add(DD a, DD b) {
  double sh, sl, th, tl, vh, vl, zh, zl;
  two_sum(a.x[0], b.x[0], sh, sl);
  two_sum(a.x[1], b.x[1], th, tl);
  double c = sl + th;
  fast_two_sum(sh, c, vh, vl);
  double w = tl + vl;
  fast_two_sum(vh, w, zh, zl);
  return dd_make(zh, zl);
}
static inline DD neg(DD a) { return dd_make(-a.x[0], -a.x[1]); }
static inline DD sub(DD a, DD b) { return add(a, neg(b)); }

// Double-word x double-word with FMA (Joldes-Muller-Popescu 2017, Alg. 12);
// relative error below 4u^2.
static inline DD mul(DD a, DD b) {
  double ch, cl1;
  two_prod(a.x[0], b.x[0], ch, cl1);
  double tl0 = a.x[1] * b.x[1];
  double tl1 = std::fma(a.x[0], b.x[1], tl0);
  double cl2 = std::fma(a.x[1], b.x[0], tl1);
  double cl3 = cl1 + cl2;
  double zh, zl;
  fast_two_sum(ch, cl3, zh, zl);
  return dd_make(zh, zl);
}

// Long division: three quotient digits, each the FP64 quotient of the
// current dd remainder's leading limb by the divisor's leading limb.
static inline DD div_(DD a, DD b) {
  double q1 = a.x[0] / b.x[0];
  DD r = sub(a, mul(b, dd_make(q1, 0.0)));
  double q2 = r.x[0] / b.x[0];
  r = sub(r, mul(b, dd_make(q2, 0.0)));
  double q3 = r.x[0] / b.x[0];
  double s, e;
  fast_two_sum(q1, q2, s, e);
  return add(dd_make(s, e), dd_make(q3, 0.0));
}

// One Newton correction of the FP64 square root: x1 = x0 + (a - x0^2)/(2 x0)
// with the residual a - x0^2 formed in dd from the exact product x0*x0.
static inline DD sqrt_(DD a) {
  if (a.x[0] <= 0.0) return dd_make(std::sqrt(a.x[0]), 0.0);
  double x0 = std::sqrt(a.x[0]);
  double p, e;
  two_prod(x0, x0, p, e);
  DD r = sub(a, dd_make(p, e));
  double corr = r.x[0] / (2.0 * x0);
  double zh, zl;
  fast_two_sum(x0, corr, zh, zl);
  return dd_make(zh, zl);
}
static inline bool is_zero(DD a) { return a.x[0] == 0.0; }
static inline bool is_finite(DD a) { return std::isfinite(a.x[0]) && std::isfinite(a.x[1]); }
static inline double hi(DD a) { return a.x[0]; }

// ------------------------------------------------------------ expansions ----
// An expansion is an array of doubles whose exact sum is the represented
// value; kept nonoverlapping and ordered by increasing magnitude, zero
// components eliminated (Shewchuk 1997).

// h := e + b exactly.  h may alias e.  Returns the new length.
static inline int exp_grow(const double *e, int n, double b, double *h) {
  double q = b;
  int k = 0;
  for (int i = 0; i < n; ++i) {
    double s, err;
    two_sum(q, e[i], s, err);
    q = s;
    if (err != 0.0) h[k++] = err;
  }
  if (q != 0.0 || k == 0) h[k++] = q;
  return k;
}
// Floating-point approximation of the value of an expansion: the sum from
// the smallest component up, then one correction with the exact remainder.
static inline double exp_approx(const double *e, int n, double *scratch) {
  double a = 0.0;
  for (int i = 0; i < n; ++i) a += e[i];
  int m = exp_grow(e, n, -a, scratch);
  double c = 0.0;
  for (int i = 0; i < m; ++i) c += scratch[i];
  return a + c;
}
// Round an expansion to `nl` limbs by successive extraction of the leading
// double: limb_k = fl(value - limb_0 - ... - limb_{k-1}), the remainder being
// kept exact.  Limbs satisfy |x_{k+1}| <= ulp(x_k) (half an ulp barring ties).
static inline void exp_round(const double *e, int n, double *out, int nl) {
  double cur[512], scr[512];
  std::memcpy(cur, e, sizeof(double) * n);
  for (int k = 0; k < nl; ++k) {
    double a = (n > 0) ? exp_approx(cur, n, scr) : 0.0;
    out[k] = a;
    if (a != 0.0) n = exp_grow(cur, n, -a, cur);
    if (n == 1 && cur[0] == 0.0) n = 0;
  }
}

// ------------------------------------------------------------------- qd ----
struct QD {
  double x[4];
};
static inline QD qd_make(double a) { QD r; r.x[0] = a; r.x[1] = r.x[2] = r.x[3] = 0.0; return r; }

static inline int qd_to_exp(const QD &a, double *e, int n) {
  for (int i = 0; i < 4; ++i)
    if (a.x[i] != 0.0) n = exp_grow(e, n, a.x[i], e);
  return n;
}
static inline QD exp_to_qd(const double *e, int n) {
  QD r;
  exp_round(e, n, r.x, 4);
  return r;
}
static inline QD add(QD a, QD b) {
  double e[16];
  int n = 0;
  n = qd_to_exp(a, e, n);
  n = qd_to_exp(b, e, n);
  return exp_to_qd(e, n);
}
static inline QD neg(QD a) { QD r; for (int i = 0; i < 4; ++i) r.x[i] = -a.x[i]; return r; }
static inline QD sub(QD a, QD b) { return add(a, neg(b)); }

// e := e + a*b exactly (all 16 limb products split by TwoProd).
static inline int exp_add_prod(double *e, int n, const QD &a, const QD &b) {
  for (int i = 0; i < 4; ++i) {
    if (a.x[i] == 0.0) continue;
    for (int j = 0; j < 4; ++j) {
      if (b.x[j] == 0.0) continue;
      double p, err;
      two_prod(a.x[i], b.x[j], p, err);
      n = exp_grow(e, n, p, e);
      if (err != 0.0) n = exp_grow(e, n, err, e);
    }
  }
  return n;
}
static inline QD mul(QD a, QD b) {
  double e[512];
  int n = exp_add_prod(e, 0, a, b);
  return exp_to_qd(e, n);
}
// Long division with five quotient digits against the exact remainder.
static inline QD div_(QD a, QD b) {
  double rem[512], scr[512], q[8];
  int n = qd_to_exp(a, rem, 0);
  QD nb = neg(b);
  for (int k = 0; k < 5; ++k) {
    double r = (n > 0) ? exp_approx(rem, n, scr) : 0.0;
    q[k] = r / b.x[0];
    if (q[k] == 0.0) { for (int j = k + 1; j < 5; ++j) q[j] = 0.0; break; }
    n = exp_add_prod(rem, n, qd_make(q[k]), nb);
  }
  double e[16];
  int m = 0;
  for (int k = 0; k < 5; ++k)
    if (q[k] != 0.0) m = exp_grow(e, m, q[k], e);
  return exp_to_qd(e, m);
}
// Newton iteration x <- x + (a - x^2) / (2x) with the residual formed
// exactly; three steps from the FP64 root (53 -> 106 -> 212 -> 424 bits).
static inline QD sqrt_(QD a) {
  if (a.x[0] <= 0.0) return qd_make(std::sqrt(a.x[0]));
  QD x = qd_make(std::sqrt(a.x[0]));
  for (int it = 0; it < 3; ++it) {
    double e[512];
    int n = qd_to_exp(a, e, 0);
    n = exp_add_prod(e, n, x, neg(x));
    QD r = exp_to_qd(e, n);
    QD two_x = add(x, x);
    x = add(x, div_(r, two_x));
  }
  return x;
}
static inline bool is_zero(QD a) { return a.x[0] == 0.0; }
static inline bool is_finite(QD a) {
  for (int i = 0; i < 4; ++i) if (!std::isfinite(a.x[i])) return false;
  return true;
}
static inline double hi(QD a) { return a.x[0]; }

// --------------------------------------------------------------- traits ----
template <class T> struct Limbs;
template <> struct Limbs<double> {
  static constexpr int L = 1;
  static double get(const double *p, size_t plane) { return p[0]; (void)plane; }
  static void put(double *p, size_t plane, double v) { p[0] = v; (void)plane; }
  static double from(double a) { return a; }
};
template <> struct Limbs<DD> {
  static constexpr int L = 2;
  // p points at limb 0 of the requested part; limb l sits 2*l planes further.
  static DD get(const double *p, size_t plane) { return dd_make(p[0], p[2 * plane]); }
  static void put(double *p, size_t plane, DD v) { p[0] = v.x[0]; p[2 * plane] = v.x[1]; }
  static DD from(double a) { return dd_make(a, 0.0); }
};
template <> struct Limbs<QD> {
  static constexpr int L = 4;
  static QD get(const double *p, size_t plane) {
    QD r;
    for (int l = 0; l < 4; ++l) r.x[l] = p[2 * plane * l];
    return r;
  }
  static void put(double *p, size_t plane, QD v) {
    for (int l = 0; l < 4; ++l) p[2 * plane * l] = v.x[l];
  }
  static QD from(double a) { return qd_make(a); }
};

// -------------------------------------------------------------- complex ----
template <class T> struct C {
  T re, im;
};
template <class T> static inline C<T> cadd(C<T> a, C<T> b) { return {add(a.re, b.re), add(a.im, b.im)}; }
template <class T> static inline C<T> csub(C<T> a, C<T> b) { return {sub(a.re, b.re), sub(a.im, b.im)}; }
// Textbook four-multiplication product.
template <class T> static inline C<T> cmul(C<T> a, C<T> b) {
  return {sub(mul(a.re, b.re), mul(a.im, b.im)), add(mul(a.re, b.im), mul(a.im, b.re))};
}
// conj(a) * b.
template <class T> static inline C<T> cmulc(C<T> a, C<T> b) {
  return {add(mul(a.re, b.re), mul(a.im, b.im)), sub(mul(a.re, b.im), mul(a.im, b.re))};
}
// |a|^2 as a real number.
template <class T> static inline T cabs2(C<T> a) { return add(mul(a.re, a.re), mul(a.im, a.im)); }
// a / r for real r: two real divisions.
template <class T> static inline C<T> cdivr(C<T> a, T r) { return {div_(a.re, r), div_(a.im, r)}; }
// a / b for complex b: conj(b) a / |b|^2.
template <class T> static inline C<T> cdiv(C<T> a, C<T> b) {
  T d = cabs2(b);
  C<T> nmr = cmulc(b, a);
  return {div_(nmr.re, d), div_(nmr.im, d)};
}

// Planar storage: plane p = 2*limb + part, each plane `plane` doubles long.
template <class T> static inline C<T> cload(const double *base, size_t plane, size_t off) {
  return {Limbs<T>::get(base + off, plane), Limbs<T>::get(base + plane + off, plane)};
}
template <class T> static inline void cstore(double *base, size_t plane, size_t off, C<T> v) {
  Limbs<T>::put(base + off, plane, v.re);
  Limbs<T>::put(base + plane + off, plane, v.im);
}

}  // namespace orc
