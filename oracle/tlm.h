/*
 * tlm.h -- TEST INFRASTRUCTURE ONLY: forward-mode (tangent-linear)
 * arithmetic for compiling the oracle (ora.c) a second time.
 *
 * A `dual` carries a value and ORA_TLM_K tangents.  Every operation the
 * oracle uses (+, -, *, /, sqrt, fabs, comparisons, isinf) acts on the value
 * as in plain FP64 and propagates the tangents by the chain rule; every
 * comparison and branch is taken on the value, so the compiled oracle is the
 * exact derivative of the branch the plain oracle takes (upwind choices,
 * limiter cases, max): the tangent-linear model of the discrete SIMPLE-TS
 * step, K directions at once.  The system headers the oracle includes come
 * first, then `double` is redefined to `dual` for the oracle's source only.
 */
#ifndef ORA_TLM_H
#define ORA_TLM_H

#include <math.h>
#include <omp.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#ifndef ORA_TLM_K
#define ORA_TLM_K 16
#endif

typedef double ora_f64;

struct dual {
  ora_f64 v;
  ora_f64 d[ORA_TLM_K];
  dual() = default;
  dual(ora_f64 x) : v(x) {
    for (int k = 0; k < ORA_TLM_K; k++) d[k] = 0.0;
  }
  dual(int x) : dual((ora_f64)x) {}
  dual(long x) : dual((ora_f64)x) {}
  dual(unsigned long x) : dual((ora_f64)x) {}
  explicit operator int() const { return (int)v; }
};

static inline dual operator+(const dual &a, const dual &b) {
  dual r;
  r.v = a.v + b.v;
  for (int k = 0; k < ORA_TLM_K; k++) r.d[k] = a.d[k] + b.d[k];
  return r;
}
static inline dual operator-(const dual &a, const dual &b) {
  dual r;
  r.v = a.v - b.v;
  for (int k = 0; k < ORA_TLM_K; k++) r.d[k] = a.d[k] - b.d[k];
  return r;
}
static inline dual operator-(const dual &a) {
  dual r;
  r.v = -a.v;
  for (int k = 0; k < ORA_TLM_K; k++) r.d[k] = -a.d[k];
  return r;
}
static inline dual operator*(const dual &a, const dual &b) {
  dual r;
  r.v = a.v * b.v;
  for (int k = 0; k < ORA_TLM_K; k++) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
static inline dual operator/(const dual &a, const dual &b) {
  dual r;
  r.v = a.v / b.v;
  const ora_f64 ib = 1.0 / b.v;
  for (int k = 0; k < ORA_TLM_K; k++) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib;
  return r;
}
static inline dual &operator+=(dual &a, const dual &b) { return a = a + b; }
static inline dual &operator-=(dual &a, const dual &b) { return a = a - b; }
static inline dual &operator*=(dual &a, const dual &b) { return a = a * b; }
static inline dual &operator/=(dual &a, const dual &b) { return a = a / b; }
static inline bool operator>(const dual &a, const dual &b) { return a.v > b.v; }
static inline bool operator<(const dual &a, const dual &b) { return a.v < b.v; }
static inline bool operator>=(const dual &a, const dual &b) { return a.v >= b.v; }
static inline bool operator<=(const dual &a, const dual &b) { return a.v <= b.v; }
static inline bool operator==(const dual &a, const dual &b) { return a.v == b.v; }
static inline bool operator!=(const dual &a, const dual &b) { return a.v != b.v; }
static inline dual sqrt(const dual &a) {
  dual r;
  r.v = sqrt(a.v);
  const ora_f64 h = 0.5 / r.v;
  for (int k = 0; k < ORA_TLM_K; k++) r.d[k] = a.d[k] * h;
  return r;
}
static inline dual fabs(const dual &a) { return a.v < 0.0 ? -a : a; }
static inline bool isinf(const dual &a) { return isinf(a.v); }

#define double dual
#endif
