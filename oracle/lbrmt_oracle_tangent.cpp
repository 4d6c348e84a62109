/*
 * lbrmt_oracle_tangent.cpp -- TEST INFRASTRUCTURE ONLY.
 *
 * The tangent-linear (forward-mode) version of the FP64 oracle: the same
 * source file, lbrmt_oracle.c, compiled as C++ with every `double` replaced by
 * a dual number (value, tangent).  Arithmetic on the value part is the
 * oracle's own, operation for operation (so the values agree with the plain
 * oracle bit for bit), and comparisons look at the value part only, so every
 * discrete decision (solid set, layers, scan windows, upwind sides, fallbacks)
 * is the one the plain oracle takes.  The tangent part is then the exact
 * derivative of that discrete map along the seeded input direction, which is
 * what a discrete adjoint of the step must reproduce.
 *
 * Derivative rules (first-order dual numbers, e^2 = 0):
 *   (a, a')(b, b') = (ab, a'b + ab'),  (a, a')/(b, b') = (a/b, (a'b - ab')/b^2),
 *   sqrt(a) -> (sqrt a, a'/(2 sqrt a)) (tangent 0 at a = 0, where the oracle
 *   only takes the root of a norm for a diagnostic), sin, cos by the chain
 *   rule, floor -> (floor a, 0).
 *
 * Only the test-suite may load the library built from this file.  The C API
 * is lbrmt_oracle.h's with `double` read as `struct { double v, d; }`.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

struct dual {
    double v, d;
    dual() = default;
    dual(double a) : v(a), d(0.0) {}
    dual(double a, double b) : v(a), d(b) {}
    explicit operator double() const { return v; }
    dual& operator+=(const dual& o) { d += o.d; v += o.v; return *this; }
    dual& operator-=(const dual& o) { d -= o.d; v -= o.v; return *this; }
    dual& operator*=(const dual& o) { *this = dual(v * o.v, d * o.v + v * o.d); return *this; }
    dual& operator/=(const dual& o);
};

static inline dual operator+(const dual& a) { return a; }
static inline dual operator-(const dual& a) { return dual(-a.v, -a.d); }
static inline dual operator+(const dual& a, const dual& b) { return dual(a.v + b.v, a.d + b.d); }
static inline dual operator-(const dual& a, const dual& b) { return dual(a.v - b.v, a.d - b.d); }
static inline dual operator*(const dual& a, const dual& b) {
    return dual(a.v * b.v, a.d * b.v + a.v * b.d);
}
static inline dual operator/(const dual& a, const dual& b) {
    double q = a.v / b.v;
    return dual(q, (a.d - q * b.d) / b.v);
}
inline dual& dual::operator/=(const dual& o) { *this = *this / o; return *this; }

static inline bool operator<(const dual& a, const dual& b) { return a.v < b.v; }
static inline bool operator>(const dual& a, const dual& b) { return a.v > b.v; }
static inline bool operator<=(const dual& a, const dual& b) { return a.v <= b.v; }
static inline bool operator>=(const dual& a, const dual& b) { return a.v >= b.v; }
static inline bool operator==(const dual& a, const dual& b) { return a.v == b.v; }
static inline bool operator!=(const dual& a, const dual& b) { return a.v != b.v; }

static inline dual sqrt(const dual& a) {
    double r = sqrt(a.v);
    return dual(r, a.v > 0.0 ? a.d / (2.0 * r) : 0.0);
}
static inline dual sin(const dual& a) { return dual(sin(a.v), cos(a.v) * a.d); }
static inline dual cos(const dual& a) { return dual(cos(a.v), -sin(a.v) * a.d); }
static inline dual floor(const dual& a) { return dual(floor(a.v), 0.0); }
static inline bool isnan(const dual& a) { return isnan(a.v); }

static_assert(sizeof(dual) == 2 * sizeof(double), "dual must be two packed doubles");

#undef _GNU_SOURCE
#define double dual
#include "lbrmt_oracle.c"
#undef double
