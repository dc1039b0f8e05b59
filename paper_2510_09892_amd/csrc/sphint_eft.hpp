// Error-free transformations and the AccuX building blocks for gfx950 (binary64 VALU).
//
// Chen, Ullrich & Panetta, "Fast and Accurate Intersections on a Sphere": Sec. 5 (accurate
// operators, Alg. 1-7) and Sec. 6 (AccuX, Alg. 8).  Every operation below is one IEEE
// binary64 rounding (round to nearest even); FMAs appear only where an algorithm asks for
// one.  Contraction is off for this whole translation unit: a compiler-fused a*b+c would
// change the rounding the error-free transformations rely on (the paper builds with
// -ffp-contract=off for the same reason, Sec. 7.2).
#pragma once
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sphint {

struct dd {
  double hi, lo;
};

// Knuth TwoSum: s = fl(a+b), e = a + b - s exactly; no precondition (6 operations).
__host__ __device__ __forceinline__ dd two_sum(double a, double b) {
  double s = a + b;
  double bv = s - a;
  double av = s - bv;
  return {s, (a - av) + (b - bv)};
}

// Dekker FastTwoSum: exact when exponent(a) >= exponent(b) (3 operations).
__host__ __device__ __forceinline__ dd fast_two_sum(double a, double b) {
  double s = a + b;
  return {s, b - (s - a)};
}

// TwoProduct with a single-rounding FMA: a*b = p + e exactly.
__host__ __device__ __forceinline__ dd two_prod(double a, double b) {
  double p = a * b;
  return {p, __builtin_fma(a, b, -p)};
}

__host__ __device__ __forceinline__ int sgn(double v) { return (v > 0.0) - (v < 0.0); }

// Alg. 4 (AccuDOP), read as a*b - c*d with compensation fl(s + fl(r1 - r2)) (the exact
// identity a*b - c*d = (p1 - p2) + (r1 - r2)), followed by a TwoSum renormalisation so that
// |lo| <= u |hi|; mag = |p1| + |p2| bounds the compensation error (3.01 u^2 mag).
struct dop3 {
  double hi, lo, mag;  // the renormalised pair and |p1| + |p2|
  bool zero;           // a*b - c*d == 0 exactly: both TwoProducts agree in both parts
};
__host__ __device__ __forceinline__ dop3 accu_dop(double a, double b, double c, double d) {
  dd p1 = two_prod(a, b);
  dd p2 = two_prod(c, d);
  dd t = two_sum(p1.hi, -p2.hi);
  double err = t.lo + (p1.lo - p2.lo);
  dd n = two_sum(t.hi, err);
  return {n.hi, n.lo, __builtin_fabs(p1.hi) + __builtin_fabs(p2.hi),
          p1.hi == p2.hi && p1.lo == p2.lo};
}

// Alg. 6 (SumNonNeg).  Its leading TwoSum adds two non-negative numbers, so it is done as
// FastTwoSum(max, min): both are exact, so the pair is the same, in fewer dependent steps.
__host__ __device__ __forceinline__ dd sum_non_neg(dd A, dd B) {
  dd H = fast_two_sum(__builtin_fmax(A.hi, B.hi), __builtin_fmin(A.hi, B.hi));
  double c = A.lo + B.lo;
  double d = H.lo + c;
  return fast_two_sum(H.hi, d);
}

// Quantities of one arc that every latitude of that arc shares (Alg. 8 lines 2-6, 13-16
// and 18-21), plus what the exact hit test needs.
struct ArcEft {
  double nx, enx, ny, eny, nz, enz;  // normal n = x1 x x2 as renormalised pairs
  double mx, my, mz;                 // AccuDOP magnitudes
  double S2, s2, S3, s3;             // |n_xy|^2 and |n|^2 as pairs (Alg. 7)
  double Fx, eFx, Fy, eFy;           // n_x n_z and n_y n_z as pairs
  double n21, n22, zz1, zz2;         // binary64 |x1|^2, |x2|^2, z1^2, z2^2 (filters only)
  double side;                       // sum |n_i| m_i (the s^2 filter's normal-error term)
  double z1, z2;
  int d1, d2;                        // exact signs of dz/dt at the endpoints
  unsigned flags;
};

// Alg. 7 (SumOfSquaresC) for the 2-D and 3-D normal at once: the 3-D sums continue the
// 2-D ones term by term, exactly as running Alg. 5 and Alg. 1 over three terms does.
__host__ __device__ __forceinline__ void norms(ArcEft& a) {
  dd st = two_prod(a.nx, a.nx);               // SumNonNeg([0,0], [P,p]) == [P,p]
  st = sum_non_neg(st, two_prod(a.ny, a.ny));  // SumOfSquares over (n_x, n_y)
  dd cp = two_prod(a.nx, a.enx);               // CompDotC over (n_x, n_y).(e_x, e_y)
  dd h = two_prod(a.ny, a.eny);
  dd q = two_sum(cp.hi, h.hi);
  double cs = cp.lo + (q.lo + h.lo);
  double cph = q.hi;
  double R2s = cph + cs;                        // CompDot
  double R2 = __builtin_fma(2.0, R2s, st.lo);
  dd S2 = fast_two_sum(st.hi, R2);
  a.S2 = S2.hi;
  a.s2 = S2.lo;
  dd st3 = sum_non_neg(st, two_prod(a.nz, a.nz));
  dd h3 = two_prod(a.nz, a.enz);
  dd q3 = two_sum(cph, h3.hi);
  double cs3 = cs + (q3.lo + h3.lo);
  double R3s = q3.hi + cs3;
  double R3 = __builtin_fma(2.0, R3s, st3.lo);
  dd S3 = fast_two_sum(st3.hi, R3);
  a.S3 = S3.hi;
  a.s3 = S3.lo;
}

// Alg. 8 lines 13-16 / 18-21: (F, e_F) = n_a n_z as a pair.
__host__ __device__ __forceinline__ dd f_pair(double na, double ena, double nz, double enz) {
  dd f = two_prod(na, nz);
  double e2 = na * enz;
  double e3 = nz * ena;
  return {f.hi, (f.lo + e2) + e3};
}

// The correctly rounded square root of a > 0.  On the GPU, for a within [2^-700, 2^700],
// the square-root sequence the compiler emits without its range steps (the reciprocal square
// root estimate and four FMA refinements; the scaling of tiny arguments and the zero and
// infinity fix-up are idle there), else the full one, as on the CPU.
__host__ __device__ __forceinline__ double sqrt_pos(double a) {
#if defined(__HIP_DEVICE_COMPILE__)
  if (a >= 0x1p-700 && a <= 0x1p700) {
    const double y = __builtin_amdgcn_rsq(a);
    double g = a * y;
    double h = y * 0.5;
    const double r = __builtin_fma(-h, g, 0.5);
    g = __builtin_fma(g, r, g);
    h = __builtin_fma(h, r, h);
    g = __builtin_fma(__builtin_fma(-g, g, a), h, g);
    return __builtin_fma(__builtin_fma(-g, g, a), h, g);
  }
#endif
  return __builtin_sqrt(a);
}

// AccSqrt of the pair (a, e), |e| <= u a: double-word square root with one first-order
// correction and a FastTwoSum renormalisation (relative error 25/8 u^2).
__host__ __device__ __forceinline__ dd acc_sqrt(double a, double e) {
  if (!(a > 0.0)) return {0.0, 0.0};
  double sh = sqrt_pos(a);
  double rho1 = __builtin_fma(-sh, sh, a);
  double rho2 = rho1 + e;
  double sl = rho2 / (2.0 * sh);
  return fast_two_sum(sh, sl);
}

// Quotients n / d over one denominator d, each the correctly rounded binary64 quotient.
// On the GPU the division sequence the compiler emits (reciprocal estimate, two Newton steps
// on the reciprocal, the product and one FMA correction) is split: its reciprocal part
// depends on d alone and runs once, and each numerator takes the product and its
// corrections (three operations instead of eleven).  The split sequence is the compiled one
// whenever that one would not rescale its operands: d and |n| within [2^-380, 2^380] keep
// the operands, the quotient and every intermediate normal with exponents less than 768
// apart.  Other operands take the ordinary division, as does the CPU build.
struct Divider {
  double d, r;
  bool ok;
};

__host__ __device__ __forceinline__ Divider divider(double d) {
  Divider v;
  v.d = d;
#if defined(__HIP_DEVICE_COMPILE__)
  v.ok = d >= 0x1p-380 && d <= 0x1p380;
  const double r0 = __builtin_amdgcn_rcp(d);
  const double r1 = __builtin_fma(r0, __builtin_fma(-d, r0, 1.0), r0);
  v.r = __builtin_fma(r1, __builtin_fma(-d, r1, 1.0), r1);
  // computed here once: without this the compiler recomputes it inside every quotient
  __asm__ volatile("" : "+v"(v.r));
#else
  v.ok = false;
  v.r = 0.0;
#endif
  return v;
}

__host__ __device__ __forceinline__ double quot(const Divider& v, double n) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double a = __builtin_fabs(n);
  if (v.ok && a >= 0x1p-380 && a <= 0x1p380) {
    const double m = n * v.r;
    return __builtin_fma(__builtin_fma(-v.d, m, n), v.r, m);
  }
#endif
  return n / v.d;
}

}  // namespace sphint
