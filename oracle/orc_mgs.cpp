// TEST INFRASTRUCTURE -- NOT PART OF THE PRODUCT PATH.
//
// CPU oracle for the complex modified Gram-Schmidt (MGS) least-squares
// solver of Verschelde and Yoffe, "Orthogonalization on a General Purpose
// Graphics Processing Unit with Double Double and Quad Double Arithmetic".
// Plain, slow, sequential definitions written from the paper:
//   * MGS, Section 3, Figure 1: for k = 1..n, r_kk = sqrt(a_k^H a_k),
//     q_k = a_k / r_kk, then for j > k: r_kj = q_k^H a_j, a_j -= r_kj q_k.
//   * Least squares, Section 3, Equation (1): MGS applied to [A b] yields
//     R, y = Q^H b and the residual column; R x = y is then solved.
//   * Back substitution, Section 6, Figure 3: column oriented, for k = n..1:
//     x_k = y_k / r_kk, then y_j -= r_jk x_k for j < k.
//   * The accuracy measure of Section 4, Equation (2).
//   * A polynomial system's values and Jacobian and Newton's method with the
//     MGS least-squares solve (Section 7: the corrector of a path tracker).
//   * The adjoint of the least-squares solution (not in the paper; the
//     differentiation form built around it): for L = Re(g^H x) with
//     x = argmin ||b - A x||, full column rank, r = b - A x and
//     z = (A^H A)^{-1} g, dL/db = A z and dL/dA = r z^H - (A z) x^H
//     (gradient convention dL/dRe + i dL/dIm).  Evaluated from the MGS
//     factors: w = R^{-H} g, z = R^{-1} w, A z = Q w.
// Every reduction runs sequentially in ascending index order.  Only the loop
// over independent trailing columns j is spread over OpenMP threads, so the
// results are bitwise identical for every thread count.
//
// Storage ("planar"): a complex matrix of `cols` columns with leading
// dimension ld is 2*L planes of ld*cols doubles; plane 2*l + part holds limb
// l of the real (part 0) or imaginary (part 1) parts, column-major.
#include "orc_arith.hpp"

#include <omp.h>

#include <cstdlib>
#include <vector>

using namespace orc;

namespace {

template <class T> using CV = std::vector<C<T>>;

template <class T> void read_planar(const double *p, int rows, int cols, int ld, CV<T> &out) {
  size_t plane = (size_t)ld * cols;
  out.resize((size_t)rows * cols);
  for (int j = 0; j < cols; ++j)
    for (int i = 0; i < rows; ++i) out[(size_t)j * rows + i] = cload<T>(p, plane, (size_t)j * ld + i);
}
template <class T> void write_planar(double *p, int rows, int cols, int ld, const CV<T> &v) {
  size_t plane = (size_t)ld * cols;
  for (int j = 0; j < cols; ++j)
    for (int i = 0; i < rows; ++i) cstore<T>(p, plane, (size_t)j * ld + i, v[(size_t)j * rows + i]);
}

template <class T> C<T> czero() { return {Limbs<T>::from(0.0), Limbs<T>::from(0.0)}; }

// x^H y over rows [0, m), ascending.
template <class T> C<T> inner(const C<T> *x, const C<T> *y, int m) {
  C<T> s = czero<T>();
  for (int i = 0; i < m; ++i) s = cadd(s, cmulc(x[i], y[i]));
  return s;
}

// MGS on the columns of W (m x ncols, column-major, overwritten by Q in its
// first n columns and by the projected remainder in columns n..ncols-1).
// Columns 0..n-1 are normalised; any further columns are only projected
// (the augmented right-hand side of Equation (1)).  R is n x ncols.
template <class T> int mgs(int m, int n, int ncols, CV<T> &W, CV<T> &R, int nthreads) {
  R.assign((size_t)n * ncols, czero<T>());
  for (int k = 0; k < n; ++k) {
    C<T> *ak = &W[(size_t)k * m];
    T s = Limbs<T>::from(0.0);
    for (int i = 0; i < m; ++i) s = add(s, cabs2(ak[i]));
    if (is_zero(s) || !is_finite(s)) return k + 1;
    T rkk = sqrt_(s);
    for (int i = 0; i < m; ++i) ak[i] = cdivr(ak[i], rkk);
    R[(size_t)k * n + k] = {rkk, Limbs<T>::from(0.0)};
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int j = k + 1; j < ncols; ++j) {
      C<T> *aj = &W[(size_t)j * m];
      C<T> r = inner(ak, aj, m);
      R[(size_t)j * n + k] = r;
      for (int i = 0; i < m; ++i) aj[i] = csub(aj[i], cmul(r, ak[i]));
    }
  }
  return 0;
}

// Figure 3, column oriented.  R is n x n with leading dimension ldr.
template <class T> void backsolve(int n, const C<T> *R, int ldr, CV<T> y, C<T> *x) {
  for (int k = n - 1; k >= 0; --k) {
    x[k] = cdivr(y[k], R[(size_t)k * ldr + k].re);
    for (int j = 0; j < k; ++j) y[j] = csub(y[j], cmul(R[(size_t)k * ldr + j], x[k]));
  }
}

template <class T>
int run_mgs(int m, int n, const double *A, int lda, const double *b, double *Q, int ldq, double *R,
            int ldr, double *y, double *rho, int nthreads) {
  int ncols = n + (b ? 1 : 0);
  CV<T> W;
  read_planar<T>(A, m, n, lda, W);
  if (b) {
    CV<T> bb;
    read_planar<T>(b, m, 1, m, bb);
    W.insert(W.end(), bb.begin(), bb.end());
  }
  CV<T> Rv;
  int info = mgs<T>(m, n, ncols, W, Rv, nthreads);
  // Q: the first n columns of W.
  CV<T> Qv(W.begin(), W.begin() + (size_t)m * n);
  write_planar<T>(Q, m, n, ldq, Qv);
  CV<T> Rn((size_t)n * n);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) Rn[(size_t)j * n + i] = Rv[(size_t)j * n + i];
  write_planar<T>(R, n, n, ldr, Rn);
  if (b) {
    CV<T> yv(Rv.begin() + (size_t)n * n, Rv.begin() + (size_t)n * n + n);
    if (y) write_planar<T>(y, n, 1, n, yv);
    if (rho) {
      // Norm of the projected right-hand side: z of Equation (1).
      T s = Limbs<T>::from(0.0);
      const C<T> *res = &W[(size_t)n * m];
      for (int i = 0; i < m; ++i) s = add(s, cabs2(res[i]));
      T z = sqrt_(s);
      const double *zp = reinterpret_cast<const double *>(&z);
      for (int l = 0; l < Limbs<T>::L; ++l) rho[l] = zp[l];
    }
  }
  return info;
}

template <class T>
int run_backsolve(int n, const double *R, int ldr, const double *y, double *x) {
  CV<T> Rv, yv;
  read_planar<T>(R, n, n, ldr, Rv);
  read_planar<T>(y, n, 1, n, yv);
  for (int k = 0; k < n; ++k)
    if (is_zero(Rv[(size_t)k * n + k].re) || !is_finite(Rv[(size_t)k * n + k].re)) return k + 1;
  CV<T> xv((size_t)n);
  backsolve<T>(n, Rv.data(), n, yv, xv.data());
  write_planar<T>(x, n, 1, n, xv);
  return 0;
}

// Section 3: y = Q^H b by sequential MGS projections of b (the same
// operations as the augmented column of Equation (1)), then Figure 3.
template <class T>
int run_ls_solve(int m, int n, const double *Q, int ldq, const double *R, int ldr, const double *b,
                 double *x) {
  CV<T> Qv, Rv, bv;
  read_planar<T>(Q, m, n, ldq, Qv);
  read_planar<T>(R, n, n, ldr, Rv);
  read_planar<T>(b, m, 1, m, bv);
  CV<T> yv((size_t)n);
  for (int k = 0; k < n; ++k) {
    const C<T> *qk = &Qv[(size_t)k * m];
    C<T> r = inner(qk, bv.data(), m);
    yv[k] = r;
    for (int i = 0; i < m; ++i) bv[i] = csub(bv[i], cmul(r, qk[i]));
  }
  for (int k = 0; k < n; ++k)
    if (is_zero(Rv[(size_t)k * n + k].re) || !is_finite(Rv[(size_t)k * n + k].re)) return k + 1;
  CV<T> xv((size_t)n);
  backsolve<T>(n, Rv.data(), n, yv, xv.data());
  write_planar<T>(x, n, 1, n, xv);
  return 0;
}

// Adjoint of the least-squares solution, closed form (see the header).
template <class T>
int run_adjoint(int m, int n, const double *A, int lda, const double *b, const double *gx, double *gA,
                double *gb, double *xo, int nthreads) {
  CV<T> W, A0, bv, gv;
  read_planar<T>(A, m, n, lda, W);
  A0 = W;
  read_planar<T>(b, m, 1, m, bv);
  read_planar<T>(gx, n, 1, n, gv);
  W.insert(W.end(), bv.begin(), bv.end());
  CV<T> Rv;
  int info = mgs<T>(m, n, n + 1, W, Rv, nthreads);
  if (info) return info;
  // x = R^{-1} y, y the last column of the augmented R
  CV<T> y(Rv.begin() + (size_t)n * n, Rv.begin() + (size_t)n * n + n);
  CV<T> x((size_t)n), w((size_t)n), z((size_t)n);
  backsolve<T>(n, Rv.data(), n, y, x.data());
  // w = R^{-H} g: w_k = (g_k - sum_{j<k} conj(r_jk) w_j) / r_kk
  for (int k = 0; k < n; ++k) {
    C<T> s = gv[k];
    for (int j = 0; j < k; ++j) s = csub(s, cmulc(Rv[(size_t)k * n + j], w[j]));
    w[k] = cdivr(s, Rv[(size_t)k * n + k].re);
  }
  backsolve<T>(n, Rv.data(), n, w, z.data());
  // bbar = Q w ; r = b - A x
  CV<T> bbar((size_t)m), r((size_t)m);
  for (int i = 0; i < m; ++i) {
    C<T> s = czero<T>();
    for (int k = 0; k < n; ++k) s = cadd(s, cmul(W[(size_t)k * m + i], w[k]));
    bbar[i] = s;
    C<T> t = bv[i];
    for (int j = 0; j < n; ++j) t = csub(t, cmul(A0[(size_t)j * m + i], x[j]));
    r[i] = t;
  }
  // Abar_ij = r_i conj(z_j) - bbar_i conj(x_j)
  CV<T> G((size_t)m * n);
  for (int j = 0; j < n; ++j) {
    C<T> zc = {z[j].re, neg(z[j].im)}, xc = {x[j].re, neg(x[j].im)};
    for (int i = 0; i < m; ++i) G[(size_t)j * m + i] = csub(cmul(r[i], zc), cmul(bbar[i], xc));
  }
  write_planar<T>(gA, m, n, m, G);
  write_planar<T>(gb, m, 1, m, bbar);
  if (xo) write_planar<T>(xo, n, 1, n, x);
  return 0;
}

// Elementwise real arithmetic probes: a, b, out hold `count` numbers of L
// limbs each, limbs of one number contiguous.
template <class T> int run_arith(int op, int count, const double *a, const double *b, double *out) {
  const int L = Limbs<T>::L;
  for (int i = 0; i < count; ++i) {
    T x, y, z;
    double *xp = reinterpret_cast<double *>(&x), *yp = reinterpret_cast<double *>(&y);
    for (int l = 0; l < L; ++l) {
      xp[l] = a[(size_t)i * L + l];
      yp[l] = b[(size_t)i * L + l];
    }
    switch (op) {
      case 0: z = add(x, y); break;
      case 1: z = sub(x, y); break;
      case 2: z = mul(x, y); break;
      case 3: z = div_(x, y); break;
      case 4: z = sqrt_(x); break;
      default: return -3;
    }
    double *zp = reinterpret_cast<double *>(&z);
    for (int l = 0; l < L; ++l) out[(size_t)i * L + l] = zp[l];
  }
  return 0;
}

// e := e + sign * a * b exactly, a and b given as L-limb arrays.
static inline int exp_add_prod_l(double *e, int n, const double *a, const double *b, int L, double sign) {
  for (int i = 0; i < L; ++i) {
    if (a[i] == 0.0) continue;
    for (int j = 0; j < L; ++j) {
      if (b[j] == 0.0) continue;
      double p, err;
      two_prod(sign * a[i], b[j], p, err);
      n = exp_grow(e, n, p, e);
      if (err != 0.0) n = exp_grow(e, n, err, e);
    }
  }
  return n;
}
static inline int exp_add_limbs(double *e, int n, const double *a, int L, double sign) {
  for (int i = 0; i < L; ++i)
    if (a[i] != 0.0) n = exp_grow(e, n, sign * a[i], e);
  return n;
}
static inline double exp_value(const double *e, int n) {
  double scr[4096];
  return n > 0 ? exp_approx(e, n, scr) : 0.0;
}

// Accuracy measures, every difference formed EXACTLY as an expansion and
// only its final value rounded to FP64:
//   out[0] = e_max of Equation (2): max_ij |a_ij - sum_l q_il r_lj|,
//   out[1] = max_j ||a_j - Q r_j||_2 / ||a_j||_2,
//   out[2] = max_lj |(Q^H Q - I)_lj|.
// Columns j are those listed in `cols` (all when cols == NULL).
// With orth == false only out[0] and out[1] are formed (out[2] = 0).
template <class T>
void run_errors(int m, int n, const double *A, int lda, const double *Q, int ldq, const double *R,
                int ldr, const int *cols, int ncols, double *out, int nthreads, bool orth_too = true) {
  const int L = Limbs<T>::L;
  CV<T> Av, Qv, Rv;
  read_planar<T>(A, m, n, lda, Av);
  read_planar<T>(Q, m, n, ldq, Qv);
  read_planar<T>(R, n, n, ldr, Rv);
  std::vector<int> js;
  if (cols)
    js.assign(cols, cols + ncols);
  else
    for (int j = 0; j < n; ++j) js.push_back(j);
  int nj = (int)js.size();
  std::vector<double> emax(nj, 0.0), bw(nj, 0.0), orth(nj, 0.0);
#pragma omp parallel for schedule(dynamic) num_threads(nthreads)
  for (int t = 0; t < nj; ++t) {
    int j = js[t];
    std::vector<double> er(4096), ei(4096);
    double e = 0.0, s2 = 0.0, a2 = 0.0;
    for (int i = 0; i < m; ++i) {
      const C<T> &a = Av[(size_t)j * m + i];
      const double *ar = reinterpret_cast<const double *>(&a.re), *ai = reinterpret_cast<const double *>(&a.im);
      int nr = exp_add_limbs(er.data(), 0, ar, L, 1.0);
      int ni = exp_add_limbs(ei.data(), 0, ai, L, 1.0);
      for (int l = 0; l <= j; ++l) {
        const C<T> &q = Qv[(size_t)l * m + i];
        const C<T> &r = Rv[(size_t)j * n + l];
        const double *qr = reinterpret_cast<const double *>(&q.re), *qi = reinterpret_cast<const double *>(&q.im);
        const double *rr = reinterpret_cast<const double *>(&r.re), *ri = reinterpret_cast<const double *>(&r.im);
        nr = exp_add_prod_l(er.data(), nr, qr, rr, L, -1.0);
        nr = exp_add_prod_l(er.data(), nr, qi, ri, L, 1.0);
        ni = exp_add_prod_l(ei.data(), ni, qr, ri, L, -1.0);
        ni = exp_add_prod_l(ei.data(), ni, qi, rr, L, -1.0);
      }
      double dr = exp_value(er.data(), nr), di = exp_value(ei.data(), ni);
      double d = std::hypot(dr, di);
      if (d > e) e = d;
      s2 += dr * dr + di * di;
      a2 += hi(a.re) * hi(a.re) + hi(a.im) * hi(a.im);
    }
    emax[t] = e;
    bw[t] = (a2 > 0) ? std::sqrt(s2 / a2) : 0.0;
    double o = 0.0;
    for (int l = 0; orth_too && l < n; ++l) {
      int nr = 0, ni = 0;
      if (l == j) { double one = 1.0; nr = exp_add_limbs(er.data(), 0, &one, 1, -1.0); }
      for (int i = 0; i < m; ++i) {
        const C<T> &x = Qv[(size_t)l * m + i];
        const C<T> &y = Qv[(size_t)j * m + i];
        const double *xr = reinterpret_cast<const double *>(&x.re), *xi = reinterpret_cast<const double *>(&x.im);
        const double *yr = reinterpret_cast<const double *>(&y.re), *yi = reinterpret_cast<const double *>(&y.im);
        // conj(x) * y = (xr yr + xi yi) + i (xr yi - xi yr)
        nr = exp_add_prod_l(er.data(), nr, xr, yr, L, 1.0);
        nr = exp_add_prod_l(er.data(), nr, xi, yi, L, 1.0);
        ni = exp_add_prod_l(ei.data(), ni, xr, yi, L, 1.0);
        ni = exp_add_prod_l(ei.data(), ni, xi, yr, L, -1.0);
      }
      double v = std::hypot(exp_value(er.data(), nr), exp_value(ei.data(), ni));
      if (v > o) o = v;
    }
    orth[t] = o;
  }
  out[0] = out[1] = out[2] = 0.0;
  for (int t = 0; t < nj; ++t) {
    if (emax[t] > out[0]) out[0] = emax[t];
    if (bw[t] > out[1]) out[1] = bw[t];
    if (orth[t] > out[2]) out[2] = orth[t];
  }
}

// Polynomial system (Section 7: the Newton corrector of a path tracker; the
// workload of the paper's Table 6): equation e is
//   f_e(x) = sum_m c_em prod_t x_{v_emt}^{d_emt},
// t over the `nvpm` variables of monomial m.  F = f(x) (neq planar) and the
// Jacobian J (neq x nvar planar, column j = d f / d x_j), every monomial and
// derivative formed as written (powers by repeated products, the other
// factors multiplied in t order), sums over m ascending.
template <class T>
void run_poly_eval(int neq, int nvar, int nmon, int nvpm, const int *vars, const int *exps, const double *coef,
                   const double *x, double *F, double *J) {
  CV<T> cv, xv;
  read_planar<T>(coef, nmon, neq, nmon, cv);  // cv[e * nmon + m]
  read_planar<T>(x, nvar, 1, nvar, xv);
  CV<T> Fv(neq, czero<T>()), Jv((size_t)neq * nvar, czero<T>());  // Jv[j * neq + e]
  const C<T> one = {Limbs<T>::from(1.0), Limbs<T>::from(0.0)};
  auto power = [&](const C<T> &b, int d) {
    C<T> r = one;
    for (int k = 0; k < d; ++k) r = cmul(r, b);
    return r;
  };
  for (int e = 0; e < neq; ++e) {
    for (int m = 0; m < nmon; ++m) {
      const int *vm = vars + ((size_t)e * nmon + m) * nvpm;
      const int *dm = exps + ((size_t)e * nmon + m) * nvpm;
      const C<T> c = cv[(size_t)e * nmon + m];
      C<T> mono = c;
      for (int t = 0; t < nvpm; ++t) mono = cmul(mono, power(xv[vm[t]], dm[t]));
      Fv[e] = cadd(Fv[e], mono);
      for (int t = 0; t < nvpm; ++t) {
        C<T> dv = cmul(c, {Limbs<T>::from((double)dm[t]), Limbs<T>::from(0.0)});
        for (int u = 0; u < nvpm; ++u)
          dv = cmul(dv, u == t ? power(xv[vm[u]], dm[u] - 1) : power(xv[vm[u]], dm[u]));
        C<T> &dst = Jv[(size_t)vm[t] * neq + e];
        dst = cadd(dst, dv);
      }
    }
  }
  write_planar<T>(F, neq, 1, neq, Fv);
  write_planar<T>(J, neq, nvar, neq, Jv);
}

// Newton's method on the system: K steps of x <- x + d, d the least-squares
// solution of J(x) d = -F(x) by MGS on [J -F] (Figure 1, Equation (1)) and
// back substitution (Figure 3).  x (nvar planar) is updated in place;
// dnorm[k] = FP64 2-norm of the k-th correction.  Returns 0 or the info of
// a failed factorisation.
template <class T>
int run_newton(int neq, int nvar, int nmon, int nvpm, const int *vars, const int *exps, const double *coef,
               double *x, int iters, double *dnorm) {
  const int L = Limbs<T>::L;
  std::vector<double> F((size_t)2 * L * neq), J((size_t)2 * L * neq * nvar);
  for (int k = 0; k < iters; ++k) {
    run_poly_eval<T>(neq, nvar, nmon, nvpm, vars, exps, coef, x, F.data(), J.data());
    for (double &v : F) v = -v;
    CV<T> W;
    read_planar<T>(J.data(), neq, nvar, neq, W);
    CV<T> bb;
    read_planar<T>(F.data(), neq, 1, neq, bb);
    W.insert(W.end(), bb.begin(), bb.end());
    CV<T> Rv;
    const int info = mgs<T>(neq, nvar, nvar + 1, W, Rv, 1);
    if (info != 0) return info;
    CV<T> y(Rv.begin() + (size_t)nvar * nvar, Rv.begin() + (size_t)nvar * nvar + nvar), d(nvar);
    backsolve<T>(nvar, Rv.data(), nvar, y, d.data());
    CV<T> xv;
    read_planar<T>(x, nvar, 1, nvar, xv);
    double s = 0.0;
    for (int j = 0; j < nvar; ++j) {
      xv[j] = cadd(xv[j], d[j]);
      s += hi(d[j].re) * hi(d[j].re) + hi(d[j].im) * hi(d[j].im);
    }
    write_planar<T>(x, nvar, 1, nvar, xv);
    if (dnorm) dnorm[k] = std::sqrt(s);
  }
  return 0;
}

int threads_or_default(int t) { return t > 0 ? t : omp_get_max_threads(); }

// ------------------------------------------------------ precision form ----
// Not in the paper: the refinement built around its solver.  Written from
// its definition:
//   1. [fl64(A) fl64(b)] is factored in FP64 by blocked MGS with panels of
//      `block` columns: inside a panel, MGS as in Figure 1; every later
//      column a_j (b included) then takes the panel's inner products
//      w_kj = q_k^H a_j, all from the same a_j, and a_j -= q_k w_kj for k
//      ascending.  y = the projections of b; x0 = R^{-1} y (Figure 3).
//   2. Repeat: r = b - A x with A, b, x widened exactly to qd and every
//      operation in qd; d = the FP64 solve of fl64(r): the panels'
//      projections replayed on r (per panel w = Q_p^H r, all from the same
//      r, then r -= q_k w_k for k ascending), then R^{-1} w; x += d.
//      Stop when ||d|| <= tol ||x|| (converged); when ||d|| > ||d_prev|| / 2
//      (stalled: that d is not applied; converged if the last applied
//      ||d|| / ||x|| <= sqrt(tol), stagnated otherwise); or after max_iter
//      steps.  Norms are FP64 2-norms of d and of the leading limbs of x.
static inline QD widen(double a) { return qd_make(a); }
static inline QD widen(const DD &a) {
  QD r;
  r.x[0] = a.x[0];
  r.x[1] = a.x[1];
  r.x[2] = r.x[3] = 0.0;
  return r;
}
static inline QD widen(const QD &a) { return a; }
template <class T> static inline C<QD> cwiden(const C<T> &a) { return {widen(a.re), widen(a.im)}; }

template <class T>
int run_refine(int m, int n, const double *A, int lda, const double *b, double *x_out, double *x0_out, int block,
               double tol, int max_iter, int *iters, double *err_est, int nthreads) {
  using D = double;
  CV<T> Av, bv;
  read_planar<T>(A, m, n, lda, Av);
  read_planar<T>(b, m, 1, m, bv);
  // 1. FP64 blocked MGS of [fl64(A) fl64(b)].
  CV<D> W((size_t)m * (n + 1));
  for (size_t e = 0; e < (size_t)m * n; ++e) W[e] = {hi(Av[e].re), hi(Av[e].im)};
  for (int i = 0; i < m; ++i) W[(size_t)n * m + i] = {hi(bv[i].re), hi(bv[i].im)};
  CV<D> R((size_t)n * (n + 1), czero<D>());  // R[j * n + k]: row k of column j
  for (int k0 = 0; k0 < n; k0 += block) {
    const int k1 = k0 + block < n ? k0 + block : n;
    for (int k = k0; k < k1; ++k) {
      C<D> *ak = &W[(size_t)k * m];
      D s = 0.0;
      for (int i = 0; i < m; ++i) s = add(s, cabs2(ak[i]));
      if (is_zero(s) || !is_finite(s)) return k + 1;
      const D rkk = sqrt_(s);
      for (int i = 0; i < m; ++i) ak[i] = cdivr(ak[i], rkk);
      R[(size_t)k * n + k] = {rkk, 0.0};
      for (int j = k + 1; j < k1; ++j) {
        C<D> *aj = &W[(size_t)j * m];
        const C<D> r = inner(ak, aj, m);
        R[(size_t)j * n + k] = r;
        for (int i = 0; i < m; ++i) aj[i] = csub(aj[i], cmul(r, ak[i]));
      }
    }
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int j = k1; j <= n; ++j) {
      C<D> *aj = &W[(size_t)j * m];
      for (int k = k0; k < k1; ++k) R[(size_t)j * n + k] = inner(&W[(size_t)k * m], aj, m);
      for (int k = k0; k < k1; ++k) {
        const C<D> *qk = &W[(size_t)k * m];
        const C<D> w = R[(size_t)j * n + k];
        for (int i = 0; i < m; ++i) aj[i] = csub(aj[i], cmul(w, qk[i]));
      }
    }
  }
  CV<D> y(R.begin() + (size_t)n * n, R.begin() + (size_t)n * n + n);
  CV<D> x64(n);
  backsolve<D>(n, R.data(), n, y, x64.data());
  CV<T> x(n);
  for (int j = 0; j < n; ++j) x[j] = {Limbs<T>::from(x64[j].re), Limbs<T>::from(x64[j].im)};
  if (x0_out) write_planar<T>(x0_out, n, 1, n, x);
  // 2. Refinement.
  int status = 0;  // 0 running, 1 converged, 2 stagnated
  int it_done = 0;
  double dprev = INFINITY, est = INFINITY;
  CV<D> r64(m), wv(n), d(n);
  for (int it = 1; it <= max_iter && status == 0; ++it) {
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int i = 0; i < m; ++i) {
      C<QD> ri = cwiden(bv[i]);
      for (int j = 0; j < n; ++j) ri = csub(ri, cmul(cwiden(Av[(size_t)j * m + i]), cwiden(x[j])));
      r64[i] = {hi(ri.re), hi(ri.im)};
    }
    for (int k0 = 0; k0 < n; k0 += block) {
      const int k1 = k0 + block < n ? k0 + block : n;
      for (int k = k0; k < k1; ++k) wv[k] = inner(&W[(size_t)k * m], r64.data(), m);
      for (int k = k0; k < k1; ++k) {
        const C<D> *qk = &W[(size_t)k * m];
        for (int i = 0; i < m; ++i) r64[i] = csub(r64[i], cmul(wv[k], qk[i]));
      }
    }
    backsolve<D>(n, R.data(), n, wv, d.data());
    double dn = 0.0, xn = 0.0;
    for (int j = 0; j < n; ++j) {
      dn += d[j].re * d[j].re + d[j].im * d[j].im;
      xn += hi(x[j].re) * hi(x[j].re) + hi(x[j].im) * hi(x[j].im);
    }
    dn = std::sqrt(dn);
    xn = std::sqrt(xn);
    if (it > 1 && dn > 0.5 * dprev) {
      status = est <= std::sqrt(tol) ? 1 : 2;
      break;
    }
    for (int j = 0; j < n; ++j) {
      x[j].re = add(x[j].re, Limbs<T>::from(d[j].re));
      x[j].im = add(x[j].im, Limbs<T>::from(d[j].im));
    }
    it_done = it;
    est = xn > 0.0 ? dn / xn : dn;
    dprev = dn;
    if (dn <= tol * xn) status = 1;
  }
  write_planar<T>(x_out, n, 1, n, x);
  if (iters) *iters = it_done;
  if (err_est) *err_est = est;
  return status == 1 ? 0 : (status == 2 ? -1 : -2);
}

}  // namespace

extern "C" {

// prec: limbs per real number, 1 (double), 2 (dd) or 4 (qd).
// A: m x n planar, lda >= m.  b: m planar (ld m) or NULL.
// Q: m x n planar (ldq).  R: n x n planar (ldr >= n), lower triangle zero.
// y: n planar (written when b != NULL).  rho: L limbs of the norm z of the
// projected right-hand side (when b != NULL).  Returns 0, k>0 when column k
// had a zero or non-finite norm, or <0 for bad arguments.
int orc_mgs(int prec, int m, int n, const double *A, int lda, const double *b, double *Q, int ldq,
            double *R, int ldr, double *y, double *rho, int nthreads) {
  if (n < 1 || m < n || lda < m || ldq < m || ldr < n) return -1;
  if (!A || !Q || !R) return -2;
  int t = threads_or_default(nthreads);
  switch (prec) {
    case 1: return run_mgs<double>(m, n, A, lda, b, Q, ldq, R, ldr, y, rho, t);
    case 2: return run_mgs<DD>(m, n, A, lda, b, Q, ldq, R, ldr, y, rho, t);
    case 4: return run_mgs<QD>(m, n, A, lda, b, Q, ldq, R, ldr, y, rho, t);
  }
  return -3;
}

int orc_backsolve(int prec, int n, const double *R, int ldr, const double *y, double *x) {
  if (n < 1 || ldr < n) return -1;
  switch (prec) {
    case 1: return run_backsolve<double>(n, R, ldr, y, x);
    case 2: return run_backsolve<DD>(n, R, ldr, y, x);
    case 4: return run_backsolve<QD>(n, R, ldr, y, x);
  }
  return -3;
}

int orc_ls_solve(int prec, int m, int n, const double *Q, int ldq, const double *R, int ldr,
                 const double *b, double *x) {
  if (n < 1 || m < n || ldq < m || ldr < n) return -1;
  switch (prec) {
    case 1: return run_ls_solve<double>(m, n, Q, ldq, R, ldr, b, x);
    case 2: return run_ls_solve<DD>(m, n, Q, ldq, R, ldr, b, x);
    case 4: return run_ls_solve<QD>(m, n, Q, ldq, R, ldr, b, x);
  }
  return -3;
}

// Adjoint of x = argmin ||b - A x|| for L = Re(g^H x): gA (m x n planar,
// ld m), gb (m), and x (n, may be NULL).  Returns info of the MGS.
int orc_adjoint(int prec, int m, int n, const double *A, int lda, const double *b, const double *gx,
                double *gA, double *gb, double *x, int nthreads) {
  if (n < 1 || m < n || lda < m) return -1;
  int t = threads_or_default(nthreads);
  switch (prec) {
    case 1: return run_adjoint<double>(m, n, A, lda, b, gx, gA, gb, x, t);
    case 2: return run_adjoint<DD>(m, n, A, lda, b, gx, gA, gb, x, t);
    case 4: return run_adjoint<QD>(m, n, A, lda, b, gx, gA, gb, x, t);
  }
  return -3;
}

// op: 0 add, 1 sub, 2 mul, 3 div, 4 sqrt (of a).
int orc_arith(int prec, int op, int count, const double *a, const double *b, double *out) {
  switch (prec) {
    case 1: return run_arith<double>(op, count, a, b, out);
    case 2: return run_arith<DD>(op, count, a, b, out);
    case 4: return run_arith<QD>(op, count, a, b, out);
  }
  return -3;
}

// out[0] = e_max of Equation (2); out[1] = max_j ||a_j - Q r_j|| / ||a_j||;
// out[2] = max |(Q^H Q - I)_lj|; over the columns j in cols[0..ncols) or all.
int orc_errors(int prec, int m, int n, const double *A, int lda, const double *Q, int ldq,
               const double *R, int ldr, const int *cols, int ncols, double *out, int nthreads) {
  int t = threads_or_default(nthreads);
  switch (prec) {
    case 1: run_errors<double>(m, n, A, lda, Q, ldq, R, ldr, cols, ncols, out, t); return 0;
    case 2: run_errors<DD>(m, n, A, lda, Q, ldq, R, ldr, cols, ncols, out, t); return 0;
    case 4: run_errors<QD>(m, n, A, lda, Q, ldq, R, ldr, cols, ncols, out, t); return 0;
  }
  return -3;
}

// The precision form (see run_refine): x (n planar, prec limbs), x0 (the
// FP64 starting solution widened, or NULL), iters and err_est (or NULL).
// Returns 0 converged, -1 stagnated, -2 max_iter reached first, k > 0 zero
// or non-finite norm at column k of the FP64 factorisation, < -2 bad
// arguments.
int orc_refine(int prec, int m, int n, const double *A, int lda, const double *b, double *x, double *x0, int block,
               double tol, int max_iter, int *iters, double *err_est, int nthreads) {
  if (n < 1 || m < n || lda < m || block < 1 || max_iter < 0) return -11;
  if (!A || !b || !x) return -12;
  int t = threads_or_default(nthreads);
  switch (prec) {
    case 2: return run_refine<DD>(m, n, A, lda, b, x, x0, block, tol, max_iter, iters, err_est, t);
    case 4: return run_refine<QD>(m, n, A, lda, b, x, x0, block, tol, max_iter, iters, err_est, t);
  }
  return -13;
}

// e_max of Equation (2) for `count` systems stored back to back (system s
// at A + s*2*prec*lda*n, Q + s*2*prec*ldq*n, R + s*2*prec*ldr*n): out[s].
// Threads take whole systems; each system is evaluated as by orc_errors.
int orc_emax_batch(int prec, int count, int m, int n, const double *A, int lda, const double *Q, int ldq,
                   const double *R, int ldr, double *out, int nthreads) {
  if (count < 0 || n < 1 || m < n || lda < m || ldq < m || ldr < n) return -1;
  if (prec != 1 && prec != 2 && prec != 4) return -3;
  const size_t sa = (size_t)2 * prec * lda * n, sq = (size_t)2 * prec * ldq * n, sr = (size_t)2 * prec * ldr * n;
#pragma omp parallel for schedule(dynamic) num_threads(threads_or_default(nthreads))
  for (int s = 0; s < count; ++s) {
    double o[3];
    const double *a = A + s * sa, *q = Q + s * sq, *r = R + s * sr;
    switch (prec) {
      case 1: run_errors<double>(m, n, a, lda, q, ldq, r, ldr, nullptr, 0, o, 1, false); break;
      case 2: run_errors<DD>(m, n, a, lda, q, ldq, r, ldr, nullptr, 0, o, 1, false); break;
      default: run_errors<QD>(m, n, a, lda, q, ldq, r, ldr, nullptr, 0, o, 1, false); break;
    }
    out[s] = o[0];
  }
  return 0;
}

// F = f(x) and the Jacobian J of the polynomial system (see run_poly_eval):
// vars, exps [neq][nmon][nvpm]; coef planar (prec, 2, neq, nmon): monomial
// m of equation e at e * nmon + m; x planar (prec, 2, nvar); F planar (prec,
// 2, neq); J planar (prec, 2, nvar, neq).
int orc_poly_eval(int prec, int neq, int nvar, int nmon, int nvpm, const int *vars, const int *exps,
                  const double *coef, const double *x, double *F, double *J) {
  if (neq < 1 || nvar < 1 || nmon < 1 || nvpm < 1) return -1;
  for (size_t k = 0; k < (size_t)neq * nmon * nvpm; ++k)
    if (vars[k] < 0 || vars[k] >= nvar || exps[k] < 0) return -2;
  switch (prec) {
    case 1: run_poly_eval<double>(neq, nvar, nmon, nvpm, vars, exps, coef, x, F, J); return 0;
    case 2: run_poly_eval<DD>(neq, nvar, nmon, nvpm, vars, exps, coef, x, F, J); return 0;
    case 4: run_poly_eval<QD>(neq, nvar, nmon, nvpm, vars, exps, coef, x, F, J); return 0;
  }
  return -3;
}

// `iters` Newton steps on the polynomial system from x (updated in place);
// dnorm (iters doubles or NULL) receives the norms of the corrections.
int orc_newton(int prec, int neq, int nvar, int nmon, int nvpm, const int *vars, const int *exps,
               const double *coef, double *x, int iters, double *dnorm) {
  if (neq < nvar || nvar < 1 || nmon < 1 || nvpm < 1 || iters < 0) return -1;
  for (size_t k = 0; k < (size_t)neq * nmon * nvpm; ++k)
    if (vars[k] < 0 || vars[k] >= nvar || exps[k] < 0) return -2;
  switch (prec) {
    case 1: return run_newton<double>(neq, nvar, nmon, nvpm, vars, exps, coef, x, iters, dnorm);
    case 2: return run_newton<DD>(neq, nvar, nmon, nvpm, vars, exps, coef, x, iters, dnorm);
    case 4: return run_newton<QD>(neq, nvar, nmon, nvpm, vars, exps, coef, x, iters, dnorm);
  }
  return -3;
}

}  // extern "C"
