// Row entries of the wall-normal Galerkin matrices, evaluated on the fly in
// device code (nothing is tabulated in memory).
//
// Row k (test function phi_k), column j (trial function phi_j).
//
// Helmholtz, S + alpha B in the Dirichlet basis phi_k = T_k - T_{k+2}:
//   B_kk = pi/2 (c_k + c_{k+2}), B_{k,k+-2} = -pi/2       (appendix matrix table)
//   S_kk = 2 pi (k+1)(k+2), S_kj = 4 pi (k+1), j = k+2, k+4, ...
//   (S = -(phi_j'', phi_k): the paper refers to Shen 1995 for it; the entries
//   follow from the Chebyshev second-derivative coefficients.)
// so row k has H_{k,k-2} = hm = -alpha pi/2, H_kk = h0, H_{k,k+2} = hpp + hm
// and H_kj = hpp = 4 pi (k+1) for every j >= k+4 of the same parity.
//
// Biharmonic, Q + a A + b B in phi_k = T_k - 2(k+2)/(k+3) T_{k+2}
// + (k+1)/(k+3) T_{k+4}:
//   B: five diagonals (appendix matrix table), A = (phi_j'', phi_k): three
//   diagonals (Sec. 4), Q = (phi_j'''', phi_k): upper triangular with
//   Q_kj = p_k q_j + r_k s_j for j >= k+2 (Sec. 4, eqs. for p_k, q_j, r_k, s_j)
//   and Q_kk = 8 pi (k+1)^2 (k+2)(k+4), the value the definition gives.
//
// c_0 = 2, c_k = 1 otherwise, c_{N-1} = 2 for Gauss-Lobatto quadrature.
#pragma once

#include <limits.h>

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace shen {

constexpr double kPi = 3.141592653589793238462643383279502884;

__device__ __forceinline__ double ck(int k, int N, int gl) { return (k == 0 || (gl && k == N - 1)) ? 2.0 : 1.0; }

// 1/d from the hardware reciprocal estimate refined by two Newton steps
// (each roughly squares the relative error), cheaper than the IEEE divide.
__device__ __forceinline__ double fast_rcp(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = __builtin_fma(-d, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-d, r, 1.0);
  return __builtin_fma(r, e, r);
}

// ----------------------------------------------------------------- Helmholtz
struct HelmRow {
  double hm;   // H_{k,k-2}
  double h0;   // H_{k,k}
  double hpp;  // H_{k,j}, j >= k+4 ; H_{k,k+2} = hpp + hm
};

__device__ __forceinline__ HelmRow helm_row(int k, double alpha, int N, int gl) {
  const double ha = 0.5 * kPi * alpha;
  const double kk = (double)k;
  HelmRow h;
  h.hm = -ha;
  h.h0 = __builtin_fma(ha, ck(k, N, gl) + ck(k + 2, N, gl), 2.0 * kPi * ((kk + 1.0) * (kk + 2.0)));
  h.hpp = 4.0 * kPi * (kk + 1.0);
  return h;
}

// Dirichlet mass row: (B u)_k = bd0 u_k + bdo (u_{k-2} + u_{k+2})
__device__ __forceinline__ double helm_mass_diag(int k, int N, int gl) {
  return 0.5 * kPi * (ck(k, N, gl) + ck(k + 2, N, gl));
}

// ---------------------------------------------------------------- biharmonic
// Reciprocals 1/(k+m), m = -1, 1, 3, 5, 7.  A parity chain steps k by 2, so
// advancing the window costs one new division per row.
struct Recip {
  double m1, p1, p3, p5, p7;
  __device__ __forceinline__ void init(int k) {
    const double kk = (double)k;
    m1 = (k == 1) ? 0.0 : fast_rcp(kk - 1.0);  // only used for k >= 4
    p1 = fast_rcp(kk + 1.0);
    p3 = fast_rcp(kk + 3.0);
    p5 = fast_rcp(kk + 5.0);
    p7 = fast_rcp(kk + 7.0);
  }
  __device__ __forceinline__ void advance(int knew) {  // from k to knew = k + 2
    m1 = p1;
    p1 = p3;
    p3 = p5;
    p5 = p7;
    p7 = fast_rcp((double)knew + 7.0);
  }
  __device__ __forceinline__ void retreat(int knew) {  // from k to knew = k - 2
    p7 = p5;
    p5 = p3;
    p3 = p1;
    p1 = m1;
    m1 = (knew == 1) ? 0.0 : fast_rcp((double)knew - 1.0);
  }
};

// Raw matrix entries of row k.
struct BihMats {
  double Bm4, Bm2, B0, B2, B4;  // B_{k,k-4}, B_{k,k-2}, B_kk, B_{k,k+2}, B_{k,k+4}
  double Am2, A0, A2;           // A_{k,k-2}, A_kk, A_{k,k+2}
  double Q0, Q2, Q4;            // Q_kk, Q_{k,k+2}, Q_{k,k+4}
  double p, r;                  // tail generators of row k
  double q2, s2, q4, s4;        // q_{k+2}, s_{k+2}, q_{k+4}, s_{k+4}
};

__device__ __forceinline__ BihMats bih_mats(int k, int N, int gl, const Recip& R) {
  const double K = (double)k;
  const double g1 = (K + 2.0) * R.p3;  // (k+2)/(k+3)
  const double g2 = (K + 1.0) * R.p3;  // (k+1)/(k+3)
  BihMats m;
  m.B0 = 0.5 * kPi * (ck(k, N, gl) + 4.0 * g1 * g1 + ck(k + 4, N, gl) * g2 * g2);
  m.B2 = -kPi * (g1 + (K + 4.0) * R.p5 * g2);
  m.B4 = 0.5 * kPi * g2;
  // B_{k,k-2} = B_{k-2,k}: -pi (k/(k+1) + (k+2)(k-1)/((k+3)(k+1)))
  m.Bm2 = (k >= 2) ? -kPi * (K * R.p1 + (K + 2.0) * (K - 1.0) * R.p3 * R.p1) : 0.0;
  // B_{k,k-4} = B_{k-4,k}: pi/2 (k-3)/(k-1)
  m.Bm4 = (k >= 4) ? 0.5 * kPi * (K - 3.0) * R.m1 : 0.0;
  m.A0 = -4.0 * kPi * (K + 1.0) * (K + 2.0) * g1;
  m.A2 = 2.0 * kPi * (K + 1.0) * (K + 2.0);
  m.Am2 = (k >= 2) ? 2.0 * kPi * (K - 1.0) * (K + 2.0) : 0.0;
  m.p = 8.0 * kPi * K * (K + 1.0) * (K + 2.0) * (K + 4.0);
  m.r = 24.0 * kPi * (K + 1.0) * (K + 2.0);
  m.q2 = R.p5;
  m.s2 = (K + 4.0) * (K + 4.0) * R.p5;
  m.q4 = R.p7;
  m.s4 = (K + 6.0) * (K + 6.0) * R.p7;
  m.Q0 = 8.0 * kPi * (K + 1.0) * (K + 1.0) * (K + 2.0) * (K + 4.0);
  m.Q2 = m.p * m.q2 + m.r * m.s2;
  m.Q4 = m.p * m.q4 + m.r * m.s4;
  return m;
}

struct BihRow {
  double hm4, hm2, h0, hp2, hp4;  // H_{k,k-4} .. H_{k,k+4}
  double p, r;                    // tail: H_kj = p q_j + r s_j, j >= k+6
  double q2, s2, q4, s4;
};

// Row k of the system from its coefficient-free entries m = bih_mats(k, ...).
__device__ __forceinline__ BihRow bih_row_from(const BihMats& m, double a, double b) {
  BihRow h;
  h.hm4 = b * m.Bm4;
  h.hm2 = a * m.Am2 + b * m.Bm2;
  h.h0 = m.Q0 + a * m.A0 + b * m.B0;
  h.hp2 = m.Q2 + a * m.A2 + b * m.B2;
  h.hp4 = m.Q4 + b * m.B4;
  h.p = m.p;
  h.r = m.r;
  h.q2 = m.q2;
  h.s2 = m.s2;
  h.q4 = m.q4;
  h.s4 = m.s4;
  return h;
}
__device__ __forceinline__ BihRow bih_row(int k, double a, double b, int N, int gl, const Recip& R) {
  return bih_row_from(bih_mats(k, N, gl, R), a, b);
}

// Coefficient-free constants of biharmonic row k, from which BihRow is
// assembled together with a few constants of rows k-2 and k-4 (the entries
// below the diagonal are those of the symmetric B above it, and q_{k+2},
// s_{k+2} are q4, s4 of row k-2).  Tabulated once per work group; every
// kernel that restarts a factorisation from another kernel's state must
// assemble its rows from the same values.  Valid for k >= -4 (only q4, s4
// are meaningful for k < 0).
struct BihConst {
  double Am2, Q0, A0, B0, A2, B2, B4, p, r, q4, s4;
};
static constexpr int kBihConstN = 11;

// The entries of row k that are polynomials in k (no division): A_{k,k-2},
// Q_kk, A_{k,k+2} and the tail generators p_k, r_k.
struct BihPoly {
  double Am2, Q0, A2, p, r;
};
__device__ __forceinline__ BihPoly bih_poly(int k) {
  const double K = (double)k;
  BihPoly c;
  c.A2 = 2.0 * kPi * (K + 1.0) * (K + 2.0);
  c.Am2 = (k >= 2) ? 2.0 * kPi * (K - 1.0) * (K + 2.0) : 0.0;
  c.p = 8.0 * kPi * K * (K + 1.0) * (K + 2.0) * (K + 4.0);
  c.r = 24.0 * kPi * (K + 1.0) * (K + 2.0);
  c.Q0 = 8.0 * kPi * (K + 1.0) * (K + 1.0) * (K + 2.0) * (K + 4.0);
  return c;
}

__device__ __forceinline__ BihConst bih_const(int k, int N, int gl) {
  const double K = (double)k;
  const double p3 = fast_rcp(K + 3.0), p5 = fast_rcp(K + 5.0), p7 = fast_rcp(K + 7.0);
  const double g1 = (K + 2.0) * p3;  // (k+2)/(k+3)
  const double g2 = (K + 1.0) * p3;  // (k+1)/(k+3)
  const BihPoly q = bih_poly(k);
  BihConst c;
  c.B0 = 0.5 * kPi * (ck(k, N, gl) + 4.0 * g1 * g1 + ck(k + 4, N, gl) * g2 * g2);
  c.B2 = -kPi * (g1 + (K + 4.0) * p5 * g2);
  c.B4 = 0.5 * kPi * g2;
  c.A0 = -4.0 * kPi * (K + 1.0) * (K + 2.0) * g1;
  c.A2 = q.A2;
  c.Am2 = q.Am2;
  c.p = q.p;
  c.r = q.r;
  c.q4 = p7;
  c.s4 = (K + 6.0) * (K + 6.0) * p7;
  c.Q0 = q.Q0;
  return c;
}

// Row k from its constants c and the needed constants of rows k-2 (B2, q4,
// s4) and k-4 (B4).
__device__ __forceinline__ BihRow bih_row_tab(int k, double a, double b, const BihConst& c, double B2m2, double q4m2,
                                              double s4m2, double B4m4) {
  (void)k;  // the row index is carried by the table entries
  // explicit fused multiply-adds: the same rounding wherever a row is built
  BihRow h;
  // rows 0 .. 3: B4m4 (k < 4), B2m2 and Am2 (k < 2) are +0 (no such rows
  // or entries), so hm4, hm2 come out zero without masking
  h.hm4 = b * B4m4;
  h.hm2 = __builtin_fma(a, c.Am2, b * B2m2);
  h.h0 = __builtin_fma(b, c.B0, __builtin_fma(a, c.A0, c.Q0));
  h.q2 = q4m2;
  h.s2 = s4m2;
  h.q4 = c.q4;
  h.s4 = c.s4;
  const double Q2 = __builtin_fma(c.p, h.q2, c.r * h.s2);
  const double Q4 = __builtin_fma(c.p, h.q4, c.r * h.s4);
  h.hp2 = __builtin_fma(b, c.B2, __builtin_fma(a, c.A2, Q2));
  h.hp4 = __builtin_fma(b, c.B4, Q4);
  h.p = c.p;
  h.r = c.r;
  return h;
}

// q_j, s_j of the Q tail
__device__ __forceinline__ double q_of(int j) { return 1.0 / ((double)j + 3.0); }
__device__ __forceinline__ double s_of(int j) {
  const double jj = (double)j;
  return (jj + 2.0) * (jj + 2.0) / (jj + 3.0);
}

// ------------------------------------------------------------------ complex
template <typename T2, typename R>
__device__ __forceinline__ T2 c_fnms(R s, T2 b, T2 a) {  // a - s b
  T2 o;
  o.x = __builtin_fma(-s, b.x, a.x);
  o.y = __builtin_fma(-s, b.y, a.y);
  return o;
}
__device__ __forceinline__ float2 c_fnms(float s, float2 b, float2 a) {
  return make_float2(__builtin_fmaf(-s, b.x, a.x), __builtin_fmaf(-s, b.y, a.y));
}
__device__ __forceinline__ double2 c_fma(double s, double2 b, double2 a) {  // a + s b
  return make_double2(__builtin_fma(s, b.x, a.x), __builtin_fma(s, b.y, a.y));
}
__device__ __forceinline__ double2 c_add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 c_sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 c_mul(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
// sigma s - v: a Crank-Nicolson right-hand side from the product v = H' u and
// the scalar products s = S(h) (s == nullptr: -v)
__device__ __forceinline__ double2 rhs_combine(double2 v, double sigma, const double2* s) {
  const double2 m = make_double2(-v.x, -v.y);
  return s ? c_fma(sigma, *s, m) : m;
}
__device__ __forceinline__ double c_abs1(double2 a) { return fmax(fabs(a.x), fabs(a.y)); }
__device__ __forceinline__ double c_absf(float2 a) { return fmax(fabs((double)a.x), fabs((double)a.y)); }
__device__ __forceinline__ double2 zero2() { return make_double2(0.0, 0.0); }
// c ? a : b per component (a select of whole double2 values can be lowered
// to a stack slot addressed by the condition)
__device__ __forceinline__ double2 c_sel(bool c, double2 a, double2 b) {
  return make_double2(c ? a.x : b.x, c ? a.y : b.y);
}

// A pivot is unusable when it is zero, not finite, or numerically zero: no
// larger than 2^-40 times the magnitude of its row's entries left of and on
// the diagonal (the unpivoted LU would then grow its factors by 2^40 or more,
// far beyond the FP64 accuracy it is meant to deliver).  Scale: |H_kk| plus
// the subdiagonal entries of row k.
constexpr double kPivTiny = 0x1p-40;
__device__ __forceinline__ bool bad_pivot(double d, double scale) { return !(fabs(d) > kPivTiny * scale) || !isfinite(d); }
// The first unusable row: rows come in increasing k, so the lowest k flagged
// so far (INT_MAX: none).  Branch-free, unlike a conditional assignment.
__device__ __forceinline__ int first_bad(int bad, bool isbad, int k) { return min(bad, isbad ? k : INT_MAX); }
__device__ __forceinline__ double row_scale(const HelmRow& h) { return fabs(h.h0) + fabs(h.hm); }
__device__ __forceinline__ double row_scale(const BihRow& h) { return fabs(h.h0) + fabs(h.hm2) + fabs(h.hm4); }

// Right-hand side of one Crank-Nicolson step (Sec. 3, eqs. ufin and gfin) in
// the scaling of the solves (the systems divided by nu dt/2, -nu dt/2).  With
// inv = 2/(nu dt) and K2 the squared wavenumber:
//   Helmholtz:  rhs = (2/nu) S(h) - (S + alpha' B) g,        alpha' = K2 - inv
//   biharmonic: rhs = (-2/nu) S(h) - (Q + a' A + b' B) u,    a' = inv - 2 K2,
//                                                           b' = K2 (K2 - inv)
// (2/(nu dt) (2B - Hbar) = -(S + alpha' B) and -2/(nu dt) (2A - 2 K2 B - Hchk)
// = -(Q + a' A + b' B) for the matrices of eqs. Helmholtz_matrix and
// Biharmonic_matrix.)
__device__ __forceinline__ double rhs_alpha(double K2, double inv) { return K2 - inv; }
__device__ __forceinline__ double rhs_a(double K2, double inv) { return __builtin_fma(-2.0, K2, inv); }
__device__ __forceinline__ double rhs_b(double K2, double inv) { return K2 * (K2 - inv); }

// Stopping rule of the FP64-residual refinement, shared by every mixed
// kernel.  After solve number `it` (0: the first FP32 solve, then one per
// correction) with correction size dmax and iterate size umax:
//  * a non-finite correction stops the iteration unconverged (FP64 re-solve);
//  * it_max == 0 asks for the uncorrected FP32 solution: accepted as it is;
//  * dmax <= tol umax: converged;
//  * a correction that fails to halve marks the rounding floor, where the
//    corrections are noise of about the size of the error left: accepted
//    when it is at most max(tol, 5e-13) umax (inside the 1e-12 target), else
//    unconverged (an ill-conditioned system whose floor lies higher);
//  * otherwise the iteration goes on (the caller stops after it_max).
constexpr double kStagTol = 5e-13;
__device__ __forceinline__ void refine_decide(int it, int it_max, double dmax, double umax, double& prev, double tol,
                                              bool& running, bool& conv) {
  if (!(dmax <= 1e300)) {
    running = false;
  } else if (it_max == 0) {
    running = false;
    conv = true;
  } else if (dmax <= tol * umax) {
    running = false;
    conv = true;
  } else if (it > 0 && dmax > 0.5 * prev) {
    running = false;
    conv = dmax <= fmax(tol, kStagTol) * umax;
  }
  prev = dmax;
}

}  // namespace shen
