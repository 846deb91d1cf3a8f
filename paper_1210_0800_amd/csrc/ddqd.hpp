// Device arithmetic for the MGS kernels: double-double (dd, 2 FP64 limbs)
// and quad-double (qd, 4 FP64 limbs) complex numbers (paper, Section 1:
// extended precision as unevaluated sums of hardware doubles, after Dekker
// 1971 and Priest 1992; Section 4 for the complex cost).
//
// Everything is built from three error-free transformations: TwoSum
// (Knuth), FastTwoSum (Dekker) and TwoProd through the hardware FMA.  All
// code must be compiled with -ffp-contract=off so that each + - * is
// rounded on its own.
//
// The hot operations are fused rather than composed from scalar dd ops:
//  * inner-product accumulation keeps, per real component, the exact running
//    sum S of the leading limb products (TwoProd + TwoSum) and one FP64 word
//    C that gathers every lower-order term: the TwoProd and TwoSum errors and
//    the hi*lo cross products.  (S, C) is renormalised once, after the
//    reduction.  Error per component below about (2k+6) u^2 sum|q_i||a_i|
//    for k terms, u = 2^-53: the classical inner-product bound in twice the
//    working precision.
//  * the column update a - r q forms the two leading products exactly,
//    sums them into a_hi with TwoSum and collects the rest in one word;
//    error below about 8 u^2 (|a| + |r||q|), the classical axpy bound.
// qd numbers use level-structured sums: terms of magnitude ~u^k |x| are
// added at level k with TwoSum, the carries moved to level k+1, level 3 is
// summed in plain FP64, and a two-pass TwoSum distillation renormalises.
// Error below a small multiple of 2^-209 relative to the operands.
#pragma once
#include <hip/hip_runtime.h>

namespace mgsq {

// ------------------------------------------------------------------ EFTs --
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  double v = s - a;
  e = (a - (s - v)) + (b - v);
}
// Exact when exponent(a) >= exponent(b).
__device__ __forceinline__ void fast_two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  e = b - (s - a);
}
__device__ __forceinline__ void two_prod(double a, double b, double &p, double &e) {
  p = a * b;
  e = __fma_rn(a, b, -p);
}

// --------------------------------------------------------------------- dd --
struct dd {
  double h, l;
};
struct cdd {
  dd re, im;
};

// Accurate dd + dd: both limb pairs summed exactly, carries folded in twice.
__device__ __forceinline__ dd dd_add(dd a, dd b) {
  double s, e, t, f;
  two_sum(a.h, b.h, s, e);
  two_sum(a.l, b.l, t, f);
  e += t;
  fast_two_sum(s, e, s, e);
  e += f;
  fast_two_sum(s, e, s, e);
  return {s, e};
}
// dd * dd: exact leading product, both cross terms through FMA.
__device__ __forceinline__ dd dd_mul(dd a, dd b) {
  double p, e;
  two_prod(a.h, b.h, p, e);
  e = __fma_rn(a.h, b.l, e);
  e = __fma_rn(a.l, b.h, e);
  fast_two_sum(p, e, p, e);
  return {p, e};
}
// 1/b by one Newton step from the FP64 reciprocal: x + x (1 - b x).
__device__ __forceinline__ dd dd_recip(dd b) {
  double x = 1.0 / b.h;
  // residual 1 - b x formed with FMA: exact for the hi limb
  double r = __fma_rn(-b.h, x, 1.0);
  r = __fma_rn(-b.l, x, r);
  double s, e;
  fast_two_sum(x, x * r, s, e);
  return {s, e};
}
// sqrt(s) for s > 0 by one Newton step of the FP64 square root:
// x + (s - x^2) / (2x), the residual from the exact square of x.
__device__ __forceinline__ dd dd_sqrt(dd s) {
  double x = sqrt(s.h);
  double p, e;
  two_prod(x, x, p, e);
  double d = ((s.h - p) - e) + s.l;  // s.h - p is exact (Sterbenz)
  double hs, hl;
  fast_two_sum(x, d * (0.5 / x), hs, hl);
  return {hs, hl};
}

// sqrt(s) and 1/sqrt(s) together from one FP64 square root and one FP64
// division: the root as in dd_sqrt (0.5/x is exactly half of 1/x), the
// inverse by one Newton step on the dd root started from 1/x, so the two
// results share their slow operations instead of chaining them.
__device__ __forceinline__ void dd_sqrt_recip(dd s, dd &root, dd &inv) {
  const double x = sqrt(s.h);
  const double y = 1.0 / x;
  double p, e;
  two_prod(x, x, p, e);
  const double d = ((s.h - p) - e) + s.l;
  fast_two_sum(x, d * (0.5 * y), root.h, root.l);
  double r = __fma_rn(-root.h, y, 1.0);
  r = __fma_rn(-root.l, y, r);
  fast_two_sum(y, y * r, inv.h, inv.l);
}

// ------------------------------------------------------------------- qd --
struct qd {
  double x0, x1, x2, x3;
};
struct cqd {
  qd re, im;
};

// Error-free two-pass distillation of four terms of decreasing magnitude
// into four limbs: the bottom-up TwoSum chain yields the leading double and
// three exact remainders, which are distilled again the same way.
__device__ __forceinline__ qd qd_renorm(double a0, double a1, double a2, double a3) {
  double s, e1, e2, e3, y0;
  two_sum(a2, a3, s, e3);
  two_sum(a1, s, s, e2);
  two_sum(a0, s, y0, e1);
  double f1, f2, y1;
  two_sum(e2, e3, s, f2);
  two_sum(e1, s, y1, f1);
  double y2, y3;
  two_sum(f1, f2, y2, y3);
  return {y0, y1, y2, y3};
}

__device__ __forceinline__ qd qd_add(qd a, qd b) {
  double s0, e0, s1, e1, s2, e2, s3, e3;
  two_sum(a.x0, b.x0, s0, e0);
  two_sum(a.x1, b.x1, s1, e1);
  two_sum(a.x2, b.x2, s2, e2);
  two_sum(a.x3, b.x3, s3, e3);
  // level 1: s1 + e0
  double t1, c1;
  two_sum(s1, e0, t1, c1);
  // level 2: s2 + e1 + c1
  double t2, c2, c3;
  two_sum(s2, e1, t2, c2);
  two_sum(t2, c1, t2, c3);
  // level 3 in FP64
  double t3 = ((s3 + e2) + (c2 + c3)) + e3;
  return qd_renorm(s0, t1, t2, t3);
}
__device__ __forceinline__ qd qd_neg(qd a) { return {-a.x0, -a.x1, -a.x2, -a.x3}; }
__device__ __forceinline__ qd qd_sub(qd a, qd b) { return qd_add(a, qd_neg(b)); }

__device__ __forceinline__ qd qd_mul(qd a, qd b) {
  // level 0 / 1 / 2 products split exactly
  double p00, q00, p01, q01, p10, q10, p02, q02, p11, q11, p20, q20;
  two_prod(a.x0, b.x0, p00, q00);
  two_prod(a.x0, b.x1, p01, q01);
  two_prod(a.x1, b.x0, p10, q10);
  two_prod(a.x0, b.x2, p02, q02);
  two_prod(a.x1, b.x1, p11, q11);
  two_prod(a.x2, b.x0, p20, q20);
  // level 1
  double s1, r1, r2;
  two_sum(p01, p10, s1, r1);
  two_sum(s1, q00, s1, r2);
  // level 2
  double s2, u1, u2, u3, u4, u5, u6;
  two_sum(p02, p11, s2, u1);
  two_sum(s2, p20, s2, u2);
  two_sum(s2, q01, s2, u3);
  two_sum(s2, q10, s2, u4);
  two_sum(s2, r1, s2, u5);
  two_sum(s2, r2, s2, u6);
  // level 3 (and the level-4 products) in FP64
  double s3 = a.x1 * b.x3;
  s3 = __fma_rn(a.x2, b.x2, s3);
  s3 = __fma_rn(a.x3, b.x1, s3);
  s3 = __fma_rn(a.x0, b.x3, s3);
  s3 = __fma_rn(a.x1, b.x2, s3);
  s3 = __fma_rn(a.x2, b.x1, s3);
  s3 = __fma_rn(a.x3, b.x0, s3);
  s3 += (q02 + q11) + (q20 + u1);
  s3 += (u2 + u3) + (u4 + (u5 + u6));
  return qd_renorm(p00, s1, s2, s3);
}
__device__ __forceinline__ qd qd_from(double a) { return {a, 0.0, 0.0, 0.0}; }

// 1/b: Newton iterations x <- x + x (1 - b x) from the FP64 reciprocal.
__device__ __forceinline__ qd qd_recip(qd b) {
  qd x = qd_from(1.0 / b.x0);
  const qd one = qd_from(1.0);
#pragma unroll 1
  for (int it = 0; it < 3; ++it) {
    qd r = qd_sub(one, qd_mul(b, x));
    x = qd_add(x, qd_mul(x, r));
  }
  return x;
}
// Inverse square root of s > 0 to about 2^-103, as a dd: one Newton step
// y + y (1 - s y^2) / 2 from the FP64 one, whose relative error (about
// 2^-52) it squares.  The step only needs dd precision: s enters through
// its two leading limbs, y^2 exactly (TwoProd), 1 - s y^2 is about 2^-52
// (its leading difference exact by Sterbenz), so one FP64 product of it
// with y is accurate to about 2^-105 relative to y.
__device__ __forceinline__ dd qd_rsqrt_dd(const qd &s) {
  const double y = 1.0 / sqrt(s.x0);
  double t, te;
  two_prod(y, y, t, te);
  const dd u = dd_mul({s.x0, s.x1}, {t, te});
  const double r = (1.0 - u.h) - u.l;
  dd out;
  fast_two_sum(y, 0.5 * (y * r), out.h, out.l);
  return out;
}
// One Newton step of the inverse square root in qd, from the dd one: the
// relative error goes from about 2^-103 to about 2^-206.
__device__ __forceinline__ qd qd_rsqrt(const qd &s) {
  const dd y1 = qd_rsqrt_dd(s);
  const qd y = {y1.h, y1.l, 0.0, 0.0};
  const qd r = qd_sub(qd_from(1.0), qd_mul(s, qd_mul(y, y)));
  const qd h = qd_mul(y, r);
  return qd_add(y, {0.5 * h.x0, 0.5 * h.x1, 0.5 * h.x2, 0.5 * h.x3});
}
// sqrt(s) for s > 0: the inverse square root y (qd_rsqrt), then x = s y
// corrected once by y (s - x^2) / 2, which squares the error of y again.
__device__ __forceinline__ qd qd_sqrt(qd s) {
  const qd y = qd_rsqrt(s);
  qd x = qd_mul(s, y);
  qd d = qd_sub(s, qd_mul(x, x));
  qd h = qd_mul(y, d);
  return qd_add(x, {0.5 * h.x0, 0.5 * h.x1, 0.5 * h.x2, 0.5 * h.x3});
}

// sqrt(s) and 1/sqrt(s) together: the inverse square root y of qd_sqrt
// is the reciprocal of the root up to its last bits; one Newton step of the
// reciprocal from y, y + y (1 - root y), takes it to full accuracy, in
// place of the three iterations of qd_recip started from the FP64
// reciprocal.
__device__ __forceinline__ void qd_sqrt_recip(qd s, qd &root, qd &inv) {
  const qd y = qd_rsqrt(s);
  const qd one = qd_from(1.0);
  qd x = qd_mul(s, y);
  qd d = qd_sub(s, qd_mul(x, x));
  qd h = qd_mul(y, d);
  root = qd_add(x, {0.5 * h.x0, 0.5 * h.x1, 0.5 * h.x2, 0.5 * h.x3});
  inv = qd_add(y, qd_mul(y, qd_sub(one, qd_mul(root, y))));
}

// --------------------------------------------------------- precisions ----
// A precision policy gathers what the kernels need: planar load / store,
// accumulators for inner products and norms with their wave shuffles, the
// fused column update, scaling by a real, and sqrt / reciprocal.
// Planar layout: limb l of the real / imaginary part lives in plane 2l / 2l+1.

struct PrecDD {
  static constexpr int L = 2;
  using R = dd;
  using C = cdd;
  struct Acc {
    double sr, cr, si, ci;  // exact leading sum and low-order word, re / im
  };

  __device__ static __forceinline__ C load(const double *p, size_t plane) {
    C v;
    v.re.h = p[0];
    v.im.h = p[plane];
    v.re.l = p[2 * plane];
    v.im.l = p[3 * plane];
    return v;
  }
  __device__ static __forceinline__ void store(double *p, size_t plane, const C &v) {
    p[0] = v.re.h;
    p[plane] = v.im.h;
    p[2 * plane] = v.re.l;
    p[3 * plane] = v.im.l;
  }
  __device__ static __forceinline__ C czero() { return {{0.0, 0.0}, {0.0, 0.0}}; }
  __device__ static __forceinline__ R rzero() { return {0.0, 0.0}; }
  __device__ static __forceinline__ R rfrom(double v) { return {v, 0.0}; }
  __device__ static __forceinline__ R rone() { return {1.0, 0.0}; }
  __device__ static __forceinline__ void acc_zero(Acc &a) { a.sr = a.cr = a.si = a.ci = 0.0; }

  // acc += conj(q) * a
  __device__ static __forceinline__ void acc_cmulc(Acc &acc, const C &q, const C &a) {
    double p1, e1, p2, e2, t1, t2;
    // real: qr ar + qi ai
    two_prod(q.re.h, a.re.h, p1, e1);
    two_prod(q.im.h, a.im.h, p2, e2);
    two_sum(acc.sr, p1, acc.sr, t1);
    two_sum(acc.sr, p2, acc.sr, t2);
    double c = acc.cr;
    c = __fma_rn(q.re.h, a.re.l, c);
    c = __fma_rn(q.re.l, a.re.h, c);
    c = __fma_rn(q.im.h, a.im.l, c);
    c = __fma_rn(q.im.l, a.im.h, c);
    acc.cr = c + ((e1 + e2) + (t1 + t2));
    // imag: qr ai - qi ar
    two_prod(q.re.h, a.im.h, p1, e1);
    two_prod(-q.im.h, a.re.h, p2, e2);
    two_sum(acc.si, p1, acc.si, t1);
    two_sum(acc.si, p2, acc.si, t2);
    c = acc.ci;
    c = __fma_rn(q.re.h, a.im.l, c);
    c = __fma_rn(q.re.l, a.im.h, c);
    c = __fma_rn(-q.im.h, a.re.l, c);
    c = __fma_rn(-q.im.l, a.re.h, c);
    acc.ci = c + ((e1 + e2) + (t1 + t2));
  }
  // acc += a * b (no conjugation): re a.re b.re - a.im b.im, im a.re b.im + a.im b.re
  __device__ static __forceinline__ void acc_cmul(Acc &acc, const C &a, const C &b) {
    double p1, e1, p2, e2, t1, t2;
    two_prod(a.re.h, b.re.h, p1, e1);
    two_prod(-a.im.h, b.im.h, p2, e2);
    two_sum(acc.sr, p1, acc.sr, t1);
    two_sum(acc.sr, p2, acc.sr, t2);
    double c = acc.cr;
    c = __fma_rn(a.re.h, b.re.l, c);
    c = __fma_rn(a.re.l, b.re.h, c);
    c = __fma_rn(-a.im.h, b.im.l, c);
    c = __fma_rn(-a.im.l, b.im.h, c);
    acc.cr = c + ((e1 + e2) + (t1 + t2));
    two_prod(a.re.h, b.im.h, p1, e1);
    two_prod(a.im.h, b.re.h, p2, e2);
    two_sum(acc.si, p1, acc.si, t1);
    two_sum(acc.si, p2, acc.si, t2);
    c = acc.ci;
    c = __fma_rn(a.re.h, b.im.l, c);
    c = __fma_rn(a.re.l, b.im.h, c);
    c = __fma_rn(a.im.h, b.re.l, c);
    c = __fma_rn(a.im.l, b.re.h, c);
    acc.ci = c + ((e1 + e2) + (t1 + t2));
  }
  __device__ static __forceinline__ void acc_set(Acc &acc, const C &v) {
    acc.sr = v.re.h;
    acc.cr = v.re.l;
    acc.si = v.im.h;
    acc.ci = v.im.l;
  }
  __device__ static __forceinline__ C conj(const C &v) { return {v.re, {-v.im.h, -v.im.l}}; }
  // v += (dr + i di) for FP64 dr, di
  __device__ static __forceinline__ void add_cd(C &v, double dr, double di) {
    v.re = dd_add(v.re, {dr, 0.0});
    v.im = dd_add(v.im, {di, 0.0});
  }
  __device__ static __forceinline__ C cneg(const C &v) { return {{-v.re.h, -v.re.l}, {-v.im.h, -v.im.l}}; }
  // acc.re += |a|^2
  __device__ static __forceinline__ void acc_abs2(Acc &acc, const C &a) {
    double p1, e1, p2, e2, t1, t2;
    two_prod(a.re.h, a.re.h, p1, e1);
    two_prod(a.im.h, a.im.h, p2, e2);
    two_sum(acc.sr, p1, acc.sr, t1);
    two_sum(acc.sr, p2, acc.sr, t2);
    double c = acc.cr;
    c = __fma_rn(2.0 * a.re.h, a.re.l, c);
    c = __fma_rn(2.0 * a.im.h, a.im.l, c);
    acc.cr = c + ((e1 + e2) + (t1 + t2));
  }
  __device__ static __forceinline__ void acc_merge(Acc &a, const Acc &b) {
    double t;
    two_sum(a.sr, b.sr, a.sr, t);
    a.cr = (a.cr + b.cr) + t;
    two_sum(a.si, b.si, a.si, t);
    a.ci = (a.ci + b.ci) + t;
  }
  __device__ static __forceinline__ void acc_merge_re(Acc &a, const Acc &b) {
    double t;
    two_sum(a.sr, b.sr, a.sr, t);
    a.cr = (a.cr + b.cr) + t;
  }
  __device__ static __forceinline__ Acc acc_shfl_xor(const Acc &a, int mask) {
    Acc b;
    b.sr = __shfl_xor(a.sr, mask);
    b.cr = __shfl_xor(a.cr, mask);
    b.si = __shfl_xor(a.si, mask);
    b.ci = __shfl_xor(a.ci, mask);
    return b;
  }
  __device__ static __forceinline__ Acc acc_shfl_xor_re(const Acc &a, int mask) {
    Acc b;
    b.sr = __shfl_xor(a.sr, mask);
    b.cr = __shfl_xor(a.cr, mask);
    b.si = b.ci = 0.0;
    return b;
  }
  __device__ static __forceinline__ C acc_value(const Acc &a) {
    C v;
    two_sum(a.sr, a.cr, v.re.h, v.re.l);
    two_sum(a.si, a.ci, v.im.h, v.im.l);
    return v;
  }
  __device__ static __forceinline__ R acc_value_re(const Acc &a) {
    R v;
    two_sum(a.sr, a.cr, v.h, v.l);
    return v;
  }

  // a -= r * q (complex r, q).
  //   re: a.re - r.re q.re + r.im q.im
  //   im: a.im - r.re q.im - r.im q.re
  __device__ static __forceinline__ void upd(C &a, const C &r, const C &q) {
    double p1, e1, p2, e2, s, t1, t2, c;
    two_prod(-r.re.h, q.re.h, p1, e1);
    two_prod(r.im.h, q.im.h, p2, e2);
    two_sum(a.re.h, p1, s, t1);
    two_sum(s, p2, s, t2);
    c = a.re.l;
    c = __fma_rn(-r.re.h, q.re.l, c);
    c = __fma_rn(-r.re.l, q.re.h, c);
    c = __fma_rn(r.im.h, q.im.l, c);
    c = __fma_rn(r.im.l, q.im.h, c);
    c += (e1 + e2) + (t1 + t2);
    fast_two_sum(s, c, a.re.h, a.re.l);
    two_prod(-r.re.h, q.im.h, p1, e1);
    two_prod(-r.im.h, q.re.h, p2, e2);
    two_sum(a.im.h, p1, s, t1);
    two_sum(s, p2, s, t2);
    c = a.im.l;
    c = __fma_rn(-r.re.h, q.im.l, c);
    c = __fma_rn(-r.re.l, q.im.h, c);
    c = __fma_rn(-r.im.h, q.re.l, c);
    c = __fma_rn(-r.im.l, q.re.h, c);
    c += (e1 + e2) + (t1 + t2);
    fast_two_sum(s, c, a.im.h, a.im.l);
  }
  // a * s for real s.
  __device__ static __forceinline__ C scale(const C &a, const R &s) {
    return {dd_mul(a.re, s), dd_mul(a.im, s)};
  }
  __device__ static __forceinline__ R sqrt_(const R &s) { return dd_sqrt(s); }
  __device__ static __forceinline__ R recip(const R &s) { return dd_recip(s); }
  __device__ static __forceinline__ void sqrt_recip(const R &s, R &root, R &inv) { dd_sqrt_recip(s, root, inv); }
  __device__ static __forceinline__ bool ok_norm(const R &s) {
    return s.h > 0.0 && s.h < INFINITY && s.l == s.l && fabs(s.l) < INFINITY;
  }
  __device__ static __forceinline__ void store_real(double *p, size_t stride, const R &v) {
    p[0] = v.h;
    p[stride] = v.l;
  }
};

struct PrecQD {
  static constexpr int L = 4;
  using R = qd;
  using C = cqd;
  using Acc = cqd;

  __device__ static __forceinline__ C load(const double *p, size_t plane) {
    C v;
    v.re.x0 = p[0];
    v.im.x0 = p[plane];
    v.re.x1 = p[2 * plane];
    v.im.x1 = p[3 * plane];
    v.re.x2 = p[4 * plane];
    v.im.x2 = p[5 * plane];
    v.re.x3 = p[6 * plane];
    v.im.x3 = p[7 * plane];
    return v;
  }
  __device__ static __forceinline__ void store(double *p, size_t plane, const C &v) {
    p[0] = v.re.x0;
    p[plane] = v.im.x0;
    p[2 * plane] = v.re.x1;
    p[3 * plane] = v.im.x1;
    p[4 * plane] = v.re.x2;
    p[5 * plane] = v.im.x2;
    p[6 * plane] = v.re.x3;
    p[7 * plane] = v.im.x3;
  }
  __device__ static __forceinline__ R rzero() { return {0.0, 0.0, 0.0, 0.0}; }
  __device__ static __forceinline__ R rfrom(double v) { return {v, 0.0, 0.0, 0.0}; }
  __device__ static __forceinline__ R rone() { return {1.0, 0.0, 0.0, 0.0}; }
  __device__ static __forceinline__ C czero() { return {rzero(), rzero()}; }
  __device__ static __forceinline__ void acc_zero(Acc &a) { a = czero(); }
  __device__ static __forceinline__ void acc_cmulc(Acc &acc, const C &q, const C &a) {
    acc.re = qd_add(acc.re, qd_add(qd_mul(q.re, a.re), qd_mul(q.im, a.im)));
    acc.im = qd_add(acc.im, qd_sub(qd_mul(q.re, a.im), qd_mul(q.im, a.re)));
  }
  __device__ static __forceinline__ void acc_abs2(Acc &acc, const C &a) {
    acc.re = qd_add(acc.re, qd_add(qd_mul(a.re, a.re), qd_mul(a.im, a.im)));
  }
  __device__ static __forceinline__ void acc_cmul(Acc &acc, const C &a, const C &b) {
    acc.re = qd_add(acc.re, qd_sub(qd_mul(a.re, b.re), qd_mul(a.im, b.im)));
    acc.im = qd_add(acc.im, qd_add(qd_mul(a.re, b.im), qd_mul(a.im, b.re)));
  }
  __device__ static __forceinline__ void acc_set(Acc &acc, const C &v) { acc = v; }
  __device__ static __forceinline__ C conj(const C &v) { return {v.re, qd_neg(v.im)}; }
  __device__ static __forceinline__ void add_cd(C &v, double dr, double di) {
    v.re = qd_add(v.re, qd_from(dr));
    v.im = qd_add(v.im, qd_from(di));
  }
  __device__ static __forceinline__ C cneg(const C &v) { return {qd_neg(v.re), qd_neg(v.im)}; }
  __device__ static __forceinline__ void acc_merge(Acc &a, const Acc &b) {
    a.re = qd_add(a.re, b.re);
    a.im = qd_add(a.im, b.im);
  }
  __device__ static __forceinline__ void acc_merge_re(Acc &a, const Acc &b) { a.re = qd_add(a.re, b.re); }
  __device__ static __forceinline__ qd shfl_qd(const qd &a, int mask) {
    return {__shfl_xor(a.x0, mask), __shfl_xor(a.x1, mask), __shfl_xor(a.x2, mask), __shfl_xor(a.x3, mask)};
  }
  __device__ static __forceinline__ Acc acc_shfl_xor(const Acc &a, int mask) {
    return {shfl_qd(a.re, mask), shfl_qd(a.im, mask)};
  }
  __device__ static __forceinline__ Acc acc_shfl_xor_re(const Acc &a, int mask) {
    return {shfl_qd(a.re, mask), rzero()};
  }
  __device__ static __forceinline__ C acc_value(const Acc &a) { return a; }
  __device__ static __forceinline__ R acc_value_re(const Acc &a) { return a.re; }
  __device__ static __forceinline__ void upd(C &a, const C &r, const C &q) {
    qd tr = qd_sub(qd_mul(r.re, q.re), qd_mul(r.im, q.im));
    qd ti = qd_add(qd_mul(r.re, q.im), qd_mul(r.im, q.re));
    a.re = qd_sub(a.re, tr);
    a.im = qd_sub(a.im, ti);
  }
  __device__ static __forceinline__ C scale(const C &a, const R &s) { return {qd_mul(a.re, s), qd_mul(a.im, s)}; }
  __device__ static __forceinline__ R sqrt_(const R &s) { return qd_sqrt(s); }
  __device__ static __forceinline__ R recip(const R &s) { return qd_recip(s); }
  __device__ static __forceinline__ void sqrt_recip(const R &s, R &root, R &inv) { qd_sqrt_recip(s, root, inv); }
  __device__ static __forceinline__ bool ok_norm(const R &s) {
    return s.x0 > 0.0 && s.x0 < INFINITY && fabs(s.x1) < INFINITY && fabs(s.x2) < INFINITY &&
           fabs(s.x3) < INFINITY;
  }
  __device__ static __forceinline__ void store_real(double *p, size_t stride, const R &v) {
    p[0] = v.x0;
    p[stride] = v.x1;
    p[2 * stride] = v.x2;
    p[3 * stride] = v.x3;
  }
};

// Plain complex double (FP64), for the blocked factorisation of the
// precision form: ordinary rounding, FMA where the product is fused.
struct cd {
  double re, im;
};
struct PrecD {
  static constexpr int L = 1;
  using R = double;
  using C = cd;
  struct Acc {
    double re, im;
  };
  __device__ static __forceinline__ C load(const double *p, size_t plane) { return {p[0], p[plane]}; }
  __device__ static __forceinline__ void store(double *p, size_t plane, const C &v) {
    p[0] = v.re;
    p[plane] = v.im;
  }
  __device__ static __forceinline__ C czero() { return {0.0, 0.0}; }
  __device__ static __forceinline__ R rzero() { return 0.0; }
  __device__ static __forceinline__ R rfrom(double v) { return v; }
  __device__ static __forceinline__ R rone() { return 1.0; }
  __device__ static __forceinline__ void acc_zero(Acc &a) { a.re = a.im = 0.0; }
  __device__ static __forceinline__ void acc_cmulc(Acc &acc, const C &q, const C &a) {
    acc.re = __fma_rn(q.re, a.re, acc.re);
    acc.re = __fma_rn(q.im, a.im, acc.re);
    acc.im = __fma_rn(q.re, a.im, acc.im);
    acc.im = __fma_rn(-q.im, a.re, acc.im);
  }
  __device__ static __forceinline__ void acc_cmul(Acc &acc, const C &a, const C &b) {
    acc.re = __fma_rn(a.re, b.re, acc.re);
    acc.re = __fma_rn(-a.im, b.im, acc.re);
    acc.im = __fma_rn(a.re, b.im, acc.im);
    acc.im = __fma_rn(a.im, b.re, acc.im);
  }
  __device__ static __forceinline__ void acc_abs2(Acc &acc, const C &a) {
    acc.re = __fma_rn(a.re, a.re, acc.re);
    acc.re = __fma_rn(a.im, a.im, acc.re);
  }
  __device__ static __forceinline__ void acc_set(Acc &acc, const C &v) {
    acc.re = v.re;
    acc.im = v.im;
  }
  __device__ static __forceinline__ void acc_merge(Acc &a, const Acc &b) {
    a.re += b.re;
    a.im += b.im;
  }
  __device__ static __forceinline__ void acc_merge_re(Acc &a, const Acc &b) { a.re += b.re; }
  __device__ static __forceinline__ Acc acc_shfl_xor(const Acc &a, int mask) {
    return {__shfl_xor(a.re, mask), __shfl_xor(a.im, mask)};
  }
  __device__ static __forceinline__ Acc acc_shfl_xor_re(const Acc &a, int mask) { return {__shfl_xor(a.re, mask), 0.0}; }
  __device__ static __forceinline__ C acc_value(const Acc &a) { return {a.re, a.im}; }
  __device__ static __forceinline__ R acc_value_re(const Acc &a) { return a.re; }
  __device__ static __forceinline__ C conj(const C &v) { return {v.re, -v.im}; }
  __device__ static __forceinline__ C cneg(const C &v) { return {-v.re, -v.im}; }
  // a -= r q
  __device__ static __forceinline__ void upd(C &a, const C &r, const C &q) {
    a.re = __fma_rn(-r.re, q.re, a.re);
    a.re = __fma_rn(r.im, q.im, a.re);
    a.im = __fma_rn(-r.re, q.im, a.im);
    a.im = __fma_rn(-r.im, q.re, a.im);
  }
  __device__ static __forceinline__ C scale(const C &a, const R &s) { return {a.re * s, a.im * s}; }
  __device__ static __forceinline__ R sqrt_(const R &s) { return sqrt(s); }
  __device__ static __forceinline__ R recip(const R &s) { return 1.0 / s; }
  __device__ static __forceinline__ bool ok_norm(const R &s) { return s > 0.0 && s < INFINITY; }
  __device__ static __forceinline__ void store_real(double *p, size_t stride, const R &v) { p[0] = v; }
};

// r = sqrt(s) and 1 / r (dd and qd: the fused forms that share their
// slow steps; FP64: the square root, then the division).
template <class P>
__device__ __forceinline__ void root_and_inverse(const typename P::R &s, typename P::R &root, typename P::R &inv) {
  if constexpr (P::L >= 2) {
    P::sqrt_recip(s, root, inv);
  } else {
    root = P::sqrt_(s);
    inv = P::recip(root);
  }
}

}  // namespace mgsq
