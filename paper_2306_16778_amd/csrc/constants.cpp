// Poles and residues of R_d(z) = 1/exp_d(-z) in binary128, rounded to FP64.
//
// theta_k: the d roots of the truncated Taylor polynomial exp_d (paper Sec. 2.1),
// found by the Aberth-Ehrlich simultaneous iteration in __float128 from starting
// points on the circle of radius (d!)^(1/d) (the geometric mean of the root
// moduli, since the product of the roots of exp_d is d! for even d).
// a_k = -d! / prod_{j != k} (theta_k - theta_j)  (Prop. pro:dec, eq. yoyo2), the
// formula the paper finds most accurate (Sec. 4), evaluated in binary128.
//
// Host code only; compiled with the system C++ compiler.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/expm_pfd.h"

namespace {

typedef __float128 q;

struct cq {
  q re, im;
};

inline cq add(cq a, cq b) { return {a.re + b.re, a.im + b.im}; }
inline cq sub(cq a, cq b) { return {a.re - b.re, a.im - b.im}; }
inline cq mul(cq a, cq b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
inline q norm2(cq a) { return a.re * a.re + a.im * a.im; }
inline cq divc(cq a, cq b) {
  // scaled division: both parts of b are O(1..d) here, no overflow concern,
  // but scale anyway so tiny corrections keep full precision
  q s = (b.re < 0 ? -b.re : b.re) + (b.im < 0 ? -b.im : b.im);
  cq bs = {b.re / s, b.im / s};
  cq as = {a.re / s, a.im / s};
  q den = norm2(bs);
  return {(as.re * bs.re + as.im * bs.im) / den, (as.im * bs.re - as.re * bs.im) / den};
}
inline q absq(cq a) {
  // |a| without sqrtq: ||a||_inf within a factor sqrt(2) is enough for tests of size
  q x = a.re < 0 ? -a.re : a.re, y = a.im < 0 ? -a.im : a.im;
  return x > y ? x : y;
}

// exp_d(z) and exp_d'(z) = exp_{d-1}(z) by Horner with exact 1/k! factors folded in:
// s = 1 + z/d (1 + ...), i.e. s_k = 1 + s_{k+1} z / k.
void eval_expd(int d, cq z, cq* p, cq* dp) {
  cq s = {1, 0};   // exp_d
  cq ds = {1, 0};  // exp_{d-1}
  for (int k = d; k >= 1; --k) {
    cq t = mul(s, z);
    s = {1 + t.re / k, t.im / k};
  }
  for (int k = d - 1; k >= 1; --k) {
    cq t = mul(ds, z);
    ds = {1 + t.re / k, t.im / k};
  }
  *p = s;
  *dp = ds;
}

q factorial_q(int d) {
  q f = 1;
  for (int k = 2; k <= d; ++k) f *= k;
  return f;
}

// Aberth-Ehrlich iteration on exp_d; returns false if it fails to converge.
bool roots_expd(int d, std::vector<cq>& z) {
  z.resize(d);
  // (d!)^(1/d) from a sum of logarithms: lgamma writes the global signgam, and
  // plans are created from several threads at once
  double logfact = 0.0;
  for (int k = 2; k <= d; ++k) logfact += std::log((double)k);
  const double r0 = std::exp(logfact / d);
  for (int k = 0; k < d; ++k) {
    const double ang = 2.0 * M_PI * (k + 0.5) / d + 0.25;
    z[k] = {(q)(r0 * std::cos(ang)), (q)(r0 * std::sin(ang))};
  }
  // Near a root the Horner sum cancels terms as large as e^{|z|}, so the
  // attainable relative accuracy is about 1e-34 * e^{|z|} / |exp_d'(z)|, well
  // below FP64 rounding for d <= 64 but above 1e-31.  Stop once the
  // corrections are below 1e-24 or have stopped shrinking below 1e-20.
  const q tol = (q)1e-24;
  q prev = (q)1e30;
  for (int it = 0; it < 2000; ++it) {
    q maxrel = 0;
    for (int k = 0; k < d; ++k) {
      cq p, dp;
      eval_expd(d, z[k], &p, &dp);
      cq w = divc(p, dp);  // Newton correction
      cq s = {0, 0};
      for (int j = 0; j < d; ++j)
        if (j != k) s = add(s, divc({1, 0}, sub(z[k], z[j])));
      cq den = sub({1, 0}, mul(w, s));
      cq corr = divc(w, den);
      z[k] = sub(z[k], corr);
      q rel = absq(corr) / (absq(z[k]) + 1);
      if (rel > maxrel) maxrel = rel;
    }
    const bool stalled = maxrel < (q)1e-20 && maxrel > prev * (q)0.5;
    prev = maxrel;
    if (maxrel < tol || stalled) {
      // two polishing sweeps of plain Newton
      for (int pass = 0; pass < 2; ++pass)
        for (int k = 0; k < d; ++k) {
          cq p, dp;
          eval_expd(d, z[k], &p, &dp);
          z[k] = sub(z[k], divc(p, dp));
        }
      return true;
    }
  }
  return false;
}

}  // namespace

namespace {
// The binary128 iteration takes milliseconds (2.6 ms at degree 16, 70 ms at 64)
// and every plan needs the constants of its degree: each degree is computed
// once per process and then copied (the values never change).
std::mutex cache_mu;
std::map<int, std::vector<double>> cache;  // degree -> theta (degree doubles) then a (degree doubles)

int compute_constants(int degree, double* theta, double* a);
}  // namespace

extern "C" int expm_pfd_constants(int degree, double* theta, double* a) {
  if (degree < 2 || degree > EXPM_PFD_MAX_DEGREE || (degree & 1)) return EXPM_PFD_ERR_DEGREE;
  if (!theta || !a) return EXPM_PFD_ERR_NULL;
  {
    std::lock_guard<std::mutex> lk(cache_mu);
    auto it = cache.find(degree);
    if (it != cache.end()) {
      std::copy(it->second.begin(), it->second.begin() + degree, theta);
      std::copy(it->second.begin() + degree, it->second.end(), a);
      return EXPM_PFD_OK;
    }
  }
  std::vector<double> v(2 * (size_t)degree);
  const int rc = compute_constants(degree, v.data(), v.data() + degree);
  if (rc != EXPM_PFD_OK) return rc;
  std::copy(v.begin(), v.begin() + degree, theta);
  std::copy(v.begin() + degree, v.end(), a);
  std::lock_guard<std::mutex> lk(cache_mu);
  cache.emplace(degree, std::move(v));
  return EXPM_PFD_OK;
}

namespace {
int compute_constants(int degree, double* theta, double* a) {
  const int d = degree;
  std::vector<cq> z;
  if (!roots_expd(d, z)) return EXPM_PFD_ERR_CONST;
  const q fact = factorial_q(d);
  struct pr {
    cq th, res;
  };
  std::vector<pr> keep;
  for (int k = 0; k < d; ++k) {
    cq prod = {1, 0};
    for (int j = 0; j < d; ++j)
      if (j != k) prod = mul(prod, sub(z[k], z[j]));
    cq res = divc({-fact, 0}, prod);
    if (z[k].im > 0) keep.push_back({z[k], res});
  }
  if ((int)keep.size() != d / 2) return EXPM_PFD_ERR_CONST;
  std::sort(keep.begin(), keep.end(), [](const pr& x, const pr& y) {
    if (x.th.re != y.th.re) return x.th.re < y.th.re;
    return x.th.im < y.th.im;
  });
  for (int k = 0; k < d / 2; ++k) {
    theta[2 * k] = (double)keep[k].th.re;
    theta[2 * k + 1] = (double)keep[k].th.im;
    a[2 * k] = (double)keep[k].res.re;
    a[2 * k + 1] = (double)keep[k].res.im;
  }
  return EXPM_PFD_OK;
}
}  // namespace

// Degree adapted to D significant digits (Sec. 4, Prop. prop:digit): the smallest
// even d whose bound M_1(d) + M_2(d, D) on the evaluated partial fractions'
// distance from e^x (x <= 0) is at most tol, else the even d with the smallest
// bound.  M_1(d) = 2^-d (Prop. pro:err); M_2 = (C_1 + C_2) sum_k |a_k| over all d
// residues, i.e. twice the sum over the pair representatives.
extern "C" int expm_pfd_choose_degree(double tol, int digits, int* degree, double* bound) {
  if (!degree) return EXPM_PFD_ERR_NULL;
  if (digits < 4 || digits > 34 || std::isnan(tol)) return EXPM_PFD_ERR_ARG;
  const double gamma = 0.29044;  // eq. eq:ecart
  const double eps = std::pow(10.0, 1 - digits);
  int best_d = 0;
  double best_b = 0.0;
  for (int d = 2; d <= EXPM_PFD_MAX_DEGREE; d += 2) {
    std::vector<double> th(d), a(d);
    if (int rc = expm_pfd_constants(d, th.data(), a.data())) return rc;
    double sum = 0.0;
    for (int k = 0; k < d / 2; ++k) sum += 2.0 * std::hypot(a[2 * k], a[2 * k + 1]);
    const double c1 = 2.0 * eps / (gamma * (1.0 - eps));
    const double c2 = 4.0 * d * eps / (gamma * (gamma - d * eps));  // gamma > d eps for digits >= 4
    const double b = std::ldexp(1.0, -d) + (c1 + c2) * sum;
    if (b <= tol) {
      *degree = d;
      if (bound) *bound = b;
      return 0;
    }
    if (best_d == 0 || b < best_b) {
      best_d = d;
      best_b = b;
    }
  }
  *degree = best_d;
  if (bound) *bound = best_b;
  return 1;
}
