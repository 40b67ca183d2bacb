// Double-double ("double-word") arithmetic for CDNA4, and the overload set that
// lets one kernel body run in either working precision y:
//   y = double  for FP32 input/output       (single/double pairing)
//   y = dd      for FP64 input/output       (double/double-double pairing; the
//               paper's double/quadruple pairing with a hardware-friendly y)
//
// A dd value is the unevaluated sum hi + lo with |lo| <= ulp(hi)/2; its unit
// roundoff is about 2^-104.  The building blocks are the error-free
// transformations TwoSum (Knuth), FastTwoSum (Dekker) and TwoProd via the
// fused multiply-add; add/mul follow the double-word algorithms analysed by
// Joldes, Muller and Popescu (ACM TOMS 2017).  Every fma is explicit; the
// library is compiled with -ffp-contract=off so no other contraction happens.
// The arithmetic is __host__ __device__: every operation is an IEEE binary64
// add, multiply or fused multiply-add, correctly rounded on either side, so a
// host build computes the same bits, and the error bounds stated below are
// pinned on the CPU against exact rational arithmetic.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

struct __align__(16) dd {
    double hi, lo;
};

__host__ __device__ __forceinline__ dd mk_dd(double hi, double lo) {
    dd r;
    r.hi = hi;
    r.lo = lo;
    return r;
}

__host__ __device__ __forceinline__ dd two_sum(double a, double b) {
    double s = a + b;
    double bb = s - a;
    double err = (a - (s - bb)) + (b - bb);
    return mk_dd(s, err);
}

// requires |a| >= |b| (or a == 0)
__host__ __device__ __forceinline__ dd fast_two_sum(double a, double b) {
    double s = a + b;
    return mk_dd(s, b - (s - a));
}

__host__ __device__ __forceinline__ dd two_prod(double a, double b) {
    double p = a * b;
    return mk_dd(p, fma(a, b, -p));
}

// "sloppy" sum: error <= 3u^2 (|a| + |b|) (u = 2^-53; first-order bound: the
// two roundings of the low parts, the final FastTwoSum exact), i.e. the
// result is the exact sum of a(1+d1) and b(1+d2) with |d1|, |d2| <= 3u^2 --
// the componentwise backward error that the mixed relative stability of the
// qd transforms needs.
__host__ __device__ __forceinline__ dd add(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi);
    double v = s.lo + (a.lo + b.lo);
    return fast_two_sum(s.hi, v);
}

// accurate sum: relative error <= 3u^2 (1 + O(u)) even under cancellation
// (Joldes, Muller, Popescu, accurate double-word addition)
__host__ __device__ __forceinline__ dd add_acc(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    double c = s.lo + t.hi;
    dd v = fast_two_sum(s.hi, c);
    double w = t.lo + v.lo;
    return fast_two_sum(v.hi, w);
}

__host__ __device__ __forceinline__ dd neg(dd a) { return mk_dd(-a.hi, -a.lo); }
__host__ __device__ __forceinline__ dd sub(dd a, dd b) { return add(a, neg(b)); }

// dd * dd, relative error <= 6u^2 (1 + O(u)): two roundings in the fma chain
// of the cross terms (2u^2 and 3u^2) and the dropped a.lo * b.lo (u^2)
__host__ __device__ __forceinline__ dd mul(dd a, dd b) {
    double p = a.hi * b.hi;
    double e = fma(a.hi, b.hi, -p);
    e = fma(a.hi, b.lo, e);
    e = fma(a.lo, b.hi, e);
    return fast_two_sum(p, e);
}

// dd * double, relative error <= 2u^2 (1 + O(u))
__host__ __device__ __forceinline__ dd mul(dd a, double b) {
    double p = a.hi * b;
    double e = fma(a.hi, b, -p);
    e = fma(a.lo, b, e);
    return fast_two_sum(p, e);
}

// dd / dd: quotient digit q1, exact-remainder correction q2, one more
// correction q3 (relative error <= 8u^2 (1 + O(u)): the two remainders are
// evaluated with the product and sum errors above)
__host__ __device__ __forceinline__ dd div(dd a, dd b) {
    double q1 = a.hi / b.hi;
    dd r = sub(a, mul(b, q1));
    double q2 = r.hi / b.hi;
    r = sub(r, mul(b, q2));
    double q3 = r.hi / b.hi;
    dd q = fast_two_sum(q1, q2);
    return add(q, mk_dd(q3, 0.0));
}

// --------------------------------------------------------------------------
// overload set shared by double and dd working precision
// --------------------------------------------------------------------------
__host__ __device__ __forceinline__ double y_from(double a, double) { return a; }
__host__ __device__ __forceinline__ dd y_from(double a, dd) { return mk_dd(a, 0.0); }

template <class Y> __host__ __device__ __forceinline__ Y mk_y(double hi, double lo);
template <> __host__ __device__ __forceinline__ double mk_y<double>(double hi, double lo) { return hi + lo; }
template <> __host__ __device__ __forceinline__ dd mk_y<dd>(double hi, double lo) { return mk_dd(hi, lo); }

__host__ __device__ __forceinline__ double hi_of(double a) { return a; }
__host__ __device__ __forceinline__ double hi_of(dd a) { return a.hi; }
// correctly rounded value to the nearest double of a dd (hi + lo rounded once)
__host__ __device__ __forceinline__ double to_double(double a) { return a; }
__host__ __device__ __forceinline__ double to_double(dd a) { return a.hi + a.lo; }

__host__ __device__ __forceinline__ double add(double a, double b) { return a + b; }
__host__ __device__ __forceinline__ double sub(double a, double b) { return a - b; }
__host__ __device__ __forceinline__ double neg(double a) { return -a; }
__host__ __device__ __forceinline__ double mul(double a, double b) { return a * b; }
__host__ __device__ __forceinline__ double div(double a, double b) { return a / b; }
__host__ __device__ __forceinline__ double add_acc(double a, double b) { return a + b; }

// a * b + c with one rounding in double.  In dd the product's error term is
// carried unnormalised into a sloppy sum: the error is at most
// 13u^2 |a b| + 3u^2 |c| (first order: 6u^2 |a b| from the product's fma
// chain, then the two roundings of the low-part sum), i.e. the result is the
// exact sum of (a b)(1 + d1) and c(1 + d2) with |d1| <= 13u^2, |d2| <= 3u^2 --
// a componentwise backward error of the same kind as a product followed by
// add().
__host__ __device__ __forceinline__ double mul_add(double a, double b, double c) { return fma(a, b, c); }
__host__ __device__ __forceinline__ dd mul_add(dd a, dd b, dd c) {
    const double p = a.hi * b.hi;
    double e = fma(a.hi, b.hi, -p);
    e = fma(a.hi, b.lo, e);
    e = fma(a.lo, b.hi, e);
    const dd s = two_sum(p, c.hi);
    return fast_two_sum(s.hi, s.lo + (e + c.lo));
}

// g * a - t * c: in double two roundings; in dd both products' error terms are
// carried unnormalised into one sloppy sum: error at most
// 13u^2 (|g a| + |t c|), a componentwise backward error of 13u^2 on each
// product (as for sub(mul(g, a), mul(t, c)))
__host__ __device__ __forceinline__ double mul_sub(double g, double a, double t, double c) {
    return fma(-t, c, g * a);
}
__host__ __device__ __forceinline__ dd mul_sub(dd g, dd a, dd t, dd c) {
    const double p = g.hi * a.hi;
    double e = fma(g.hi, a.hi, -p);
    e = fma(g.hi, a.lo, e);
    e = fma(g.lo, a.hi, e);
    const double q = t.hi * c.hi;
    double f = fma(t.hi, c.hi, -q);
    f = fma(t.hi, c.lo, f);
    f = fma(t.lo, c.hi, f);
    const dd s = two_sum(p, -q);
    return fast_two_sum(s.hi, s.lo + (e - f));
}

// product of the leading parts, for values needed to binary64 accuracy only
// (relative error below 3 * 2^-53 in dd)
__host__ __device__ __forceinline__ double prod_hi(double a, double b) { return a * b; }
__host__ __device__ __forceinline__ double prod_hi(dd a, dd b) { return a.hi * b.hi; }

// x * 2^k (exact unless it under/overflows)
__host__ __device__ __forceinline__ double y_ldexp(double a, int k) { return __builtin_ldexp(a, k); }
__host__ __device__ __forceinline__ dd y_ldexp(dd a, int k) {
    return mk_dd(__builtin_ldexp(a.hi, k), __builtin_ldexp(a.lo, k));
}

// binary exponent of the leading part (frexp convention: |x| in [2^(e-1), 2^e));
// 0 for x == 0
__device__ __forceinline__ int y_exp(double a) { return __builtin_amdgcn_frexp_exp(a); }
__device__ __forceinline__ int y_exp(dd a) { return __builtin_amdgcn_frexp_exp(a.hi); }

__host__ __device__ __forceinline__ bool y_neg(double a) { return a < 0.0; }
__host__ __device__ __forceinline__ bool y_neg(dd a) { return a.hi < 0.0; }

__host__ __device__ __forceinline__ double y_abs_hi(double a) { return fabs(a); }
__host__ __device__ __forceinline__ double y_abs_hi(dd a) { return fabs(a.hi); }

// unit roundoff used in thresholds
template <class Y> struct YEps;
template <> struct YEps<double> { static constexpr double v = 1.1102230246251565e-16; };
template <> struct YEps<dd> { static constexpr double v = 4.93038065763132e-32; }; // 2^-104
