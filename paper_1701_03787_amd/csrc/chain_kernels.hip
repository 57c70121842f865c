// "Chain" kernels: one lane per odd/even parity chain of one system.
//
// The Helmholtz and biharmonic matrices decouple into the even and the odd
// coefficients (Sec. 4), so every system is two independent chains.  A
// workgroup of one wavefront takes S systems: it stages their right-hand
// sides in LDS with coalesced loads, lanes 0..2S-1 each run one chain's
// O(N) recurrences sequentially against LDS (LU factors kept in LDS for
// the back substitution), and the wavefront stores the solutions with
// coalesced writes.  Simple and general in N; S is set by the LDS budget.
//
// Helmholtz per chain (upper-Hessenberg LU, Sec. 4): with h the row entries
// of shen_rows.hpp,
//   l_k = hm / d_{k-2},  d_k = h0_k - l_k (g_{k-2} + hm),  g_k = hpp_k - l_k g_{k-2}
//   y_k = f_k - l_k y_{k-2}
//   u_k = (y_k - (g_k + hm) u_{k+2} - g_k S_{k+4}) / d_k,  S_m = sum_{j>=m} u_j
// (U_{k,k+2} = g_k + hm because both entries are updated by the same l_k.)
//
// Biharmonic per chain (Alg. LUbiharmonic / ReduceAB / LUSolveBiharmonic):
// row k of U is (U0, U2, U4) on columns k, k+2, k+4 plus the tail
// P_k q_j + R_k s_j for j >= k+6, P and R playing the role of the a_k, b_k
// of ReduceAB.  Row k is reduced first by row k-4 (multiplier L2), then by
// row k-2 (multiplier L1); only these two previous rows are kept.
#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>

#include "shen_rows.hpp"
#include "shen_launch.hpp"

namespace shen {

static constexpr int kChainThreads = 64;

// ---------------------------------------------------------------------------
// shared helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int last_of_parity(int n, int p) {  // largest k < n, k%2 == p (or < 0)
  const int k = n - 1;
  return k - ((k - p) & 1);
}

__device__ __forceinline__ void load_rows(double2* __restrict__ dst, int stride_elems, const double2* __restrict__ src,
                                          int64_t w0, int Sb, int N, int n) {
  for (int s = 0; s < Sb; ++s) {
    const double2* row = src + (w0 + s) * (int64_t)N;
    double2* d = dst + s * stride_elems;
    for (int k = threadIdx.x; k < n; k += kChainThreads) d[k] = row[k];
  }
}

__device__ __forceinline__ void store_rows(double2* __restrict__ out, const double2* __restrict__ src, int stride_elems,
                                           int64_t w0, int Sb, int N, int n) {
  for (int s = 0; s < Sb; ++s) {
    double2* row = out + (w0 + s) * (int64_t)N;
    const double2* x = src + s * stride_elems;
    for (int k = threadIdx.x; k < N; k += kChainThreads) row[k] = (k < n) ? x[k] : zero2();
  }
}

// ===========================================================================
// Helmholtz
// ===========================================================================

// FP64 forward sweep: factor + y = L^{-1} f, in place in x; fac[k] = (1/d_k, g_k).
__device__ __forceinline__ int helm_fwd64(double2* x, double2* fac, int p, int n, int N, int gl, double al) {
  int bad = INT_MAX;
  double rdp = 0.0, gp = 0.0;
  double2 yp = zero2();
  for (int k = p; k < n; k += 2) {
    const HelmRow h = helm_row(k, al, N, gl);
    const double2 fk = x[k];
    double d, g;
    double2 y;
    if (k < 2) {
      d = h.h0;
      g = h.hpp;
      y = fk;
    } else {
      const double l = h.hm * rdp;
      d = __builtin_fma(-l, gp + h.hm, h.h0);
      g = __builtin_fma(-l, gp, h.hpp);
      y = c_fnms(l, yp, fk);
    }
    if (bad_pivot(d, row_scale(h)) && bad == INT_MAX) bad = k;
    const double rd = 1.0 / d;
    fac[k] = make_double2(rd, g);
    x[k] = y;
    rdp = rd;
    gp = g;
    yp = y;
  }
  return bad;
}

// FP64 back substitution with the running suffix sum, in place in x.
__device__ __forceinline__ void helm_back64(double2* x, const double2* fac, int p, int n, double hm) {
  double2 u2 = zero2(), S4 = zero2();
  for (int k = last_of_parity(n, p); k >= 0; k -= 2) {
    const double2 fr = fac[k];
    const double g = fr.y, e = g + hm;
    double2 v = c_fnms(e, u2, x[k]);
    v = c_fnms(g, S4, v);
    const double2 uk = c_mul(fr.x, v);
    x[k] = uk;
    S4 = c_add(S4, u2);
    u2 = uk;
  }
}

__device__ __forceinline__ void write_info(int32_t* info, int* bad_lds, int64_t w0, int Sb) {
  __syncthreads();
  if (info != nullptr && (int)threadIdx.x < Sb) {
    const int b = bad_lds[threadIdx.x];
    info[w0 + threadIdx.x] = (b == INT_MAX) ? 0 : b + 1;
  }
}

// Layout per system: x[NP] (double2), fac[NP] (double2); then S ints.
__global__ __launch_bounds__(kChainThreads) void helm_chain_solve(int N, int64_t nsys, int S, int NP, const double* __restrict__ alpha,
                                                                   const double2* __restrict__ f, double2* __restrict__ u,
                                                                   int gl, int32_t* __restrict__ info) {
  extern __shared__ double2 lds[];
  const int64_t w0 = (int64_t)blockIdx.x * S;
  const int Sb = (int)min((int64_t)S, nsys - w0);
  const int n = N - 2;
  const int stride = 2 * NP;
  int* bad_lds = reinterpret_cast<int*>(lds + (size_t)S * stride);
  if ((int)threadIdx.x < Sb) bad_lds[threadIdx.x] = INT_MAX;
  load_rows(lds, stride, f, w0, Sb, N, n);
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 2 * Sb) {
    const int s = t >> 1, p = t & 1;
    double2* x = lds + s * stride;
    double2* fac = x + NP;
    const double al = alpha[w0 + s];
    const int bad = helm_fwd64(x, fac, p, n, N, gl, al);
    if (bad != INT_MAX) atomicMin(&bad_lds[s], bad);
    helm_back64(x, fac, p, n, -0.5 * kPi * al);
  }
  __syncthreads();
  store_rows(u, lds, stride, w0, Sb, N, n);
  write_info(info, bad_lds, w0, Sb);
}

// Transposed solve H^T lam = g (and optional grad_alpha = -Re(lam^H B u)):
//   U^T z = g forward:  z_k = (g_k - (g_{k-2} + hm) z_{k-2} - sum_{j<=k-4} g_j z_j) / d_k
//   L^T lam = z backward: lam_k = z_k - l_{k+2} lam_{k+2}
// Layout per system: x[NP] (double2), lfac[NP] (double, l_k).
__global__ __launch_bounds__(kChainThreads) void helm_chain_adjoint(int N, int64_t nsys, int S, int NP, const double* __restrict__ alpha,
                                                                     const double2* __restrict__ ufwd, const double2* __restrict__ gbar,
                                                                     double2* __restrict__ lam_out, double* __restrict__ grad_alpha,
                                                                     int gl, int32_t* __restrict__ info) {
  extern __shared__ double2 lds[];
  const int64_t w0 = (int64_t)blockIdx.x * S;
  const int Sb = (int)min((int64_t)S, nsys - w0);
  const int n = N - 2;
  const int stride = NP + (NP + 1) / 2;  // double2 units: x[NP] then NP doubles
  int* bad_lds = reinterpret_cast<int*>(lds + (size_t)S * stride);
  if ((int)threadIdx.x < Sb) bad_lds[threadIdx.x] = INT_MAX;
  load_rows(lds, stride, gbar, w0, Sb, N, n);
  __syncthreads();
  const int t = threadIdx.x;
  double gsum = 0.0;
  if (t < 2 * Sb) {
    const int s = t >> 1, p = t & 1;
    double2* x = lds + s * stride;
    double* lf = reinterpret_cast<double*>(x + NP);
    const double al = alpha[w0 + s];
    int bad = INT_MAX;
    double rdp = 0.0, gp = 0.0;
    double2 zp = zero2(), Zacc = zero2();
    for (int k = p; k < n; k += 2) {
      const HelmRow h = helm_row(k, al, N, gl);
      double d, g, l = 0.0;
      double2 r = x[k];
      if (k < 2) {
        d = h.h0;
        g = h.hpp;
      } else {
        l = h.hm * rdp;
        d = __builtin_fma(-l, gp + h.hm, h.h0);
        g = __builtin_fma(-l, gp, h.hpp);
        r = c_fnms(gp + h.hm, zp, r);
      }
      r = c_sub(r, Zacc);
      if (bad_pivot(d, row_scale(h)) && bad == INT_MAX) bad = k;
      const double rd = 1.0 / d;
      const double2 z = c_mul(rd, r);
      x[k] = z;
      lf[k] = l;
      if (k >= 2) Zacc = c_fma(gp, zp, Zacc);
      zp = z;
      gp = g;
      rdp = rd;
    }
    if (bad != INT_MAX) atomicMin(&bad_lds[s], bad);
    const double2* uu = ufwd ? ufwd + (w0 + s) * (int64_t)N : nullptr;
    double2 lam2 = zero2();
    for (int k = last_of_parity(n, p); k >= 0; k -= 2) {
      const double l2 = (k + 2 < n) ? lf[k + 2] : 0.0;
      const double2 lam = c_fnms(l2, lam2, x[k]);
      x[k] = lam;
      lam2 = lam;
      if (uu != nullptr) {
        // (B u)_k = bd0 u_k - pi/2 (u_{k-2} + u_{k+2})
        double2 bu = c_mul(helm_mass_diag(k, N, gl), uu[k]);
        if (k >= 2) bu = c_fnms(0.5 * kPi, uu[k - 2], bu);
        if (k + 2 < n) bu = c_fnms(0.5 * kPi, uu[k + 2], bu);
        gsum -= lam.x * bu.x + lam.y * bu.y;
      }
    }
  }
  gsum += __shfl_xor(gsum, 1);
  if (t < 2 * Sb && (t & 1) == 0 && grad_alpha != nullptr && ufwd != nullptr) grad_alpha[w0 + (t >> 1)] = gsum;
  __syncthreads();
  store_rows(lam_out, lds, stride, w0, Sb, N, n);
  write_info(info, bad_lds, w0, Sb);
}

// Hu (or H^T u) with one backward / forward sweep per chain.
// Layout per system: x[NP] (double2).
// With rhs != 0 (and trans == 0): alpha holds K2 per system and the result is
// the Crank-Nicolson right-hand side sigma S(h) - (S + alpha' B) u, alpha' =
// K2 - inv (sh = S(h) rows, or null).
__global__ __launch_bounds__(kChainThreads) void helm_chain_matvec(int N, int64_t nsys, int S, int NP, const double* __restrict__ alpha,
                                                                    const double2* __restrict__ uin, double2* __restrict__ out, int gl,
                                                                    int trans, int rhs, double inv, double sigma,
                                                                    const double2* __restrict__ sh) {
  extern __shared__ double2 lds[];
  const int64_t w0 = (int64_t)blockIdx.x * S;
  const int Sb = (int)min((int64_t)S, nsys - w0);
  const int n = N - 2;
  const int stride = NP;
  load_rows(lds, stride, uin, w0, Sb, N, n);
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 2 * Sb) {
    const int s = t >> 1, p = t & 1;
    const double2* x = lds + s * stride;
    double2* o = out + (w0 + s) * (int64_t)N;
    const double2* so = sh ? sh + (w0 + s) * (int64_t)N : nullptr;
    const double al = rhs ? rhs_alpha(alpha[w0 + s], inv) : alpha[w0 + s];
    if (!trans) {
      double2 S4 = zero2(), u2 = zero2();  // S_{k+4}, u_{k+2}
      for (int k = last_of_parity(n, p); k >= 0; k -= 2) {
        const HelmRow h = helm_row(k, al, N, gl);
        const double2 uk = x[k];
        double2 v = c_mul(h.h0, uk);
        v = c_fma(h.hpp + h.hm, u2, v);
        v = c_fma(h.hpp, S4, v);
        if (k >= 2) v = c_fma(h.hm, x[k - 2], v);
        if (rhs) v = rhs_combine(v, sigma, so ? so + k : nullptr);
        o[k] = v;
        S4 = c_add(S4, u2);
        u2 = uk;
      }
    } else {
      // (H^T u)_k = H_{k-2,k} u_{k-2} + h0_k u_k + hm u_{k+2} + sum_{j<=k-4} hpp_j u_j
      double2 P = zero2();  // sum_{j<=k-4} hpp_j u_j
      double hpp_m2 = 0.0, hpp_m4 = 0.0;
      double2 um2 = zero2(), um4 = zero2();
      for (int k = p; k < n; k += 2) {
        const HelmRow h = helm_row(k, al, N, gl);
        if (k >= 4) P = c_fma(hpp_m4, um4, P);
        const double2 uk = x[k];
        double2 v = c_mul(h.h0, uk);
        if (k >= 2) v = c_fma(hpp_m2 + h.hm, um2, v);
        if (k + 2 < n) v = c_fma(h.hm, x[k + 2], v);
        v = c_add(v, P);
        o[k] = v;
        hpp_m4 = hpp_m2;
        um4 = um2;
        hpp_m2 = h.hpp;
        um2 = uk;
      }
    }
  }
  // tail zero
  for (int s = 0; s < Sb; ++s)
    for (int k = n + threadIdx.x; k < N; k += kChainThreads) out[(w0 + s) * (int64_t)N + k] = zero2();
}

// FP32 factor / solve with FP64 residual refinement.
// Layout per system (bytes): fv double2[NP] | uu double2[NP] | wk float2[NP] | fc float2[NP]
// (wk and fc together double as double2[NP] FP64 factors for the fallback).
__device__ __forceinline__ void helm_fwd32(float2* w, float2* fc, int p, int n, int N, int gl, double al, bool factor) {
  float rdp = 0.f, gp = 0.f;
  float2 yp = make_float2(0.f, 0.f);
  const float hm = (float)(-0.5 * kPi * al);
  for (int k = p; k < n; k += 2) {
    float rd, g, l = 0.f;
    if (factor) {
      const HelmRow h = helm_row(k, al, N, gl);
      float d;
      if (k < 2) {
        d = (float)h.h0;
        g = (float)h.hpp;
      } else {
        l = hm * rdp;
        d = __builtin_fmaf(-l, gp + hm, (float)h.h0);
        g = __builtin_fmaf(-l, gp, (float)h.hpp);
      }
      rd = 1.0f / d;
      fc[k] = make_float2(rd, g);
    } else {
      const float2 fr = fc[k];
      rd = fr.x;
      g = fr.y;
      l = (k < 2) ? 0.f : hm * rdp;
    }
    const float2 y = (k < 2) ? w[k] : c_fnms(l, yp, w[k]);
    w[k] = y;
    rdp = rd;
    gp = g;
    yp = y;
  }
}

// back substitution of the FP32 factors; adds the correction into uu (FP64),
// suffix sum accumulated in FP64; returns max |delta|.
__device__ __forceinline__ double helm_back32_add(const float2* w, const float2* fc, double2* uu, int p, int n, double al, bool first) {
  const float hm = (float)(-0.5 * kPi * al);
  double2 S4 = zero2();
  float2 u2 = make_float2(0.f, 0.f);
  double dmax = 0.0;
  for (int k = last_of_parity(n, p); k >= 0; k -= 2) {
    const float2 fr = fc[k];
    const float g = fr.y, e = g + hm;
    const float2 S4f = make_float2((float)S4.x, (float)S4.y);
    float2 v = c_fnms(e, u2, w[k]);
    v = c_fnms(g, S4f, v);
    const float2 dk = make_float2(fr.x * v.x, fr.x * v.y);
    const double2 dd = make_double2((double)dk.x, (double)dk.y);
    uu[k] = first ? dd : c_add(uu[k], dd);
    dmax = fmax(dmax, c_abs1(dd));
    S4 = c_add(S4, make_double2((double)u2.x, (double)u2.y));
    u2 = dk;
  }
  return dmax;
}

// r = f - H u in FP64 (backward sweep with the suffix sum), stored as complex64 in w;
// returns max |u| over the chain.
__device__ __forceinline__ double helm_residual(const double2* fv, const double2* uu, float2* w, int p, int n, int N, int gl, double al) {
  double2 S4 = zero2(), u2 = zero2();
  double umax = 0.0;
  for (int k = last_of_parity(n, p); k >= 0; k -= 2) {
    const HelmRow h = helm_row(k, al, N, gl);
    const double2 uk = uu[k];
    double2 r = c_fnms(h.h0, uk, fv[k]);
    r = c_fnms(h.hpp + h.hm, u2, r);
    r = c_fnms(h.hpp, S4, r);
    if (k >= 2) r = c_fnms(h.hm, uu[k - 2], r);
    w[k] = make_float2((float)r.x, (float)r.y);
    umax = fmax(umax, c_abs1(uk));
    S4 = c_add(S4, u2);
    u2 = uk;
  }
  return umax;
}

// every entry of one parity chain of x finite
__device__ __forceinline__ bool finite_rows(const double2* x, int p, int n) {
  bool ok = true;
  for (int k = p; k < n; k += 2) ok = ok && isfinite(x[k].x) && isfinite(x[k].y);
  return ok;
}

__global__ __launch_bounds__(kChainThreads) void helm_chain_mixed(int N, int64_t nsys, int S, int NP, const double* __restrict__ alpha,
                                                                   const double2* __restrict__ f, double2* __restrict__ u, int gl,
                                                                   int32_t* __restrict__ info, int32_t* __restrict__ iters,
                                                                   int it_max, double tol) {
  extern __shared__ double2 lds[];
  const int64_t w0 = (int64_t)blockIdx.x * S;
  const int Sb = (int)min((int64_t)S, nsys - w0);
  const int n = N - 2;
  const int stride = 3 * NP;  // double2 units: fv, uu, (wk + fc)
  int* bad_lds = reinterpret_cast<int*>(lds + (size_t)S * stride);
  if ((int)threadIdx.x < Sb) bad_lds[threadIdx.x] = INT_MAX;
  load_rows(lds, stride, f, w0, Sb, N, n);
  __syncthreads();
  const int t = threadIdx.x;
  const bool act = t < 2 * Sb;
  const int s = t >> 1, p = t & 1;
  double2* fv = lds + s * stride;
  double2* uu = fv + NP;
  float2* wk = reinterpret_cast<float2*>(uu + NP);
  float2* fc = wk + NP;
  const double al = act ? alpha[w0 + s] : 0.0;
  if (act) {
    for (int k = p; k < n; k += 2) wk[k] = make_float2((float)fv[k].x, (float)fv[k].y);
    helm_fwd32(wk, fc, p, n, N, gl, al, true);
    helm_back32_add(wk, fc, uu, p, n, al, true);
  }
  // refinement (the two lanes of a system decide together)
  bool running = act, converged = false;
  double prev = 1e300;
  int ncorr = 0;
  if (it_max == 0) {  // the uncorrected FP32 solution, when finite
    running = false;
    const int fin = (act && finite_rows(uu, p, n)) ? 1 : 0;
    converged = act && (fin & __shfl_xor(fin, 1)) != 0;
  }
  for (int it = 1; it <= it_max; ++it) {
    double umax = 0.0, dmax = 0.0;
    if (running) {
      umax = helm_residual(fv, uu, wk, p, n, N, gl, al);
      helm_fwd32(wk, fc, p, n, N, gl, al, false);
      dmax = helm_back32_add(wk, fc, uu, p, n, al, false);
      umax = fmax(umax, 0.0);
    }
    umax = fmax(umax, __shfl_xor(umax, 1));
    dmax = fmax(dmax, __shfl_xor(dmax, 1));
    if (running) {
      ncorr = it;
      refine_decide(it, it_max, dmax, umax, prev, tol, running, converged);
    }
    if (!__any(running)) break;
  }
  if (act && running) converged = false;
  if (iters != nullptr && act && p == 0) iters[w0 + s] = ncorr;
  // FP64 fallback for systems that did not converge
  if (act && !converged) {
    double2* x = uu;
    double2* fac = reinterpret_cast<double2*>(wk);
    for (int k = p; k < n; k += 2) x[k] = fv[k];
    const int bad = helm_fwd64(x, fac, p, n, N, gl, al);
    if (bad != INT_MAX) atomicMin(&bad_lds[s], bad);
    helm_back64(x, fac, p, n, -0.5 * kPi * al);
    if (bad == INT_MAX) atomicMin(&bad_lds[s], INT_MAX - 1);  // marks "fell back"
  }
  __syncthreads();
  store_rows(u, lds + NP, stride, w0, Sb, N, n);
  __syncthreads();
  if (info != nullptr && (int)threadIdx.x < Sb) {
    const int b = bad_lds[threadIdx.x];
    info[w0 + threadIdx.x] = (b == INT_MAX) ? 0 : (b == INT_MAX - 1 ? -2 : b + 1);
  }
}

// ===========================================================================
// Biharmonic
// ===========================================================================

struct BihState {  // one reduced row of U
  double rU0, U2, U4, P, R;
};

// FP64 factor + forward elimination for one chain.  If fac != null the back
// substitution factors are stored (5 arrays of NP doubles); if lfac != null the
// multipliers L1, L2 are stored (2 arrays).  Calls back `onrow` style code is
// avoided: the transposed variant has its own loop.
__device__ __forceinline__ int bih_fwd64(double2* x, double* fac, int NP, int p, int n, int N, int gl, double a, double b) {
  int bad = INT_MAX;
  BihState m2 = {0, 0, 0, 0, 0}, m4 = {0, 0, 0, 0, 0};
  double2 y2 = zero2(), y4 = zero2();
  Recip R;
  R.init(p);
  for (int k = p; k < n; k += 2) {
    if (k != p) R.advance(k);
    const BihRow h = bih_row(k, a, b, N, gl, R);
    double tm2 = h.hm2, t0 = h.h0, t2 = h.hp2, t4 = h.hp4, P = h.p, Rr = h.r;
    double2 y = x[k];
    if (k >= 4) {
      const double l2 = h.hm4 * m4.rU0;
      tm2 = __builtin_fma(-l2, m4.U2, tm2);
      t0 = __builtin_fma(-l2, m4.U4, t0);
      t2 = __builtin_fma(-l2, __builtin_fma(m4.P, h.q2, m4.R * h.s2), t2);
      t4 = __builtin_fma(-l2, __builtin_fma(m4.P, h.q4, m4.R * h.s4), t4);
      P = __builtin_fma(-l2, m4.P, P);
      Rr = __builtin_fma(-l2, m4.R, Rr);
      y = c_fnms(l2, y4, y);
    }
    if (k >= 2) {
      const double l1 = tm2 * m2.rU0;
      t0 = __builtin_fma(-l1, m2.U2, t0);
      t2 = __builtin_fma(-l1, m2.U4, t2);
      t4 = __builtin_fma(-l1, __builtin_fma(m2.P, h.q4, m2.R * h.s4), t4);
      P = __builtin_fma(-l1, m2.P, P);
      Rr = __builtin_fma(-l1, m2.R, Rr);
      y = c_fnms(l1, y2, y);
    }
    if (bad_pivot(t0, row_scale(h)) && bad == INT_MAX) bad = k;
    const double rU0 = 1.0 / t0;
    fac[k] = rU0;
    fac[NP + k] = t2;
    fac[2 * NP + k] = t4;
    fac[3 * NP + k] = P;
    fac[4 * NP + k] = Rr;
    x[k] = y;
    m4 = m2;
    y4 = y2;
    m2 = BihState{rU0, t2, t4, P, Rr};
    y2 = y;
  }
  return bad;
}

__device__ __forceinline__ void bih_back64(double2* x, const double* fac, int NP, int p, int n) {
  double2 u2 = zero2(), u4 = zero2(), sq = zero2(), ss = zero2();
  for (int k = last_of_parity(n, p); k >= 0; k -= 2) {
    double2 v = c_fnms(fac[NP + k], u2, x[k]);
    v = c_fnms(fac[2 * NP + k], u4, v);
    v = c_fnms(fac[3 * NP + k], sq, v);
    v = c_fnms(fac[4 * NP + k], ss, v);
    const double2 uk = c_mul(fac[k], v);
    x[k] = uk;
    // sums over j >= k+4 for the next row k-2
    sq = c_fma(q_of(k + 4), u4, sq);
    ss = c_fma(s_of(k + 4), u4, ss);
    u4 = u2;
    u2 = uk;
  }
}

// Layout per system: x double2[NP] | fac double[5 NP] ; then S ints.
__global__ __launch_bounds__(kChainThreads) void bih_chain_solve(int N, int64_t nsys, int S, int NP, const double* __restrict__ ca,
                                                                  const double* __restrict__ cb, const double2* __restrict__ f,
                                                                  double2* __restrict__ u, int gl, int32_t* __restrict__ info) {
  extern __shared__ double2 lds[];
  const int64_t w0 = (int64_t)blockIdx.x * S;
  const int Sb = (int)min((int64_t)S, nsys - w0);
  const int n = N - 4;
  const int stride = NP + (5 * NP + 1) / 2;
  int* bad_lds = reinterpret_cast<int*>(lds + (size_t)S * stride);
  if ((int)threadIdx.x < Sb) bad_lds[threadIdx.x] = INT_MAX;
  load_rows(lds, stride, f, w0, Sb, N, n);
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 2 * Sb) {
    const int s = t >> 1, p = t & 1;
    double2* x = lds + s * stride;
    double* fac = reinterpret_cast<double*>(x + NP);
    const int bad = bih_fwd64(x, fac, NP, p, n, N, gl, ca[w0 + s], cb[w0 + s]);
    if (bad != INT_MAX) atomicMin(&bad_lds[s], bad);
    bih_back64(x, fac, NP, p, n);
  }
  __syncthreads();
  store_rows(u, lds, stride, w0, Sb, N, n);
  write_info(info, bad_lds, w0, Sb);
}

// Transposed: U^T z = g forward (prefix sums of P_j z_j and R_j z_j, fused with
// the factorisation), then L^T lam = z backward with the stored L1, L2.
// Optional grad_a = -Re(lam^H A u), grad_b = -Re(lam^H B u).
// Layout per system: x double2[NP] | L1 double[NP] | L2 double[NP].
__global__ __launch_bounds__(kChainThreads) void bih_chain_adjoint(int N, int64_t nsys, int S, int NP, const double* __restrict__ ca,
                                                                    const double* __restrict__ cb, const double2* __restrict__ ufwd,
                                                                    const double2* __restrict__ gbar, double2* __restrict__ lam_out,
                                                                    double* __restrict__ grad_a, double* __restrict__ grad_b, int gl,
                                                                    int32_t* __restrict__ info) {
  extern __shared__ double2 lds[];
  const int64_t w0 = (int64_t)blockIdx.x * S;
  const int Sb = (int)min((int64_t)S, nsys - w0);
  const int n = N - 4;
  const int stride = 2 * NP;
  int* bad_lds = reinterpret_cast<int*>(lds + (size_t)S * stride);
  if ((int)threadIdx.x < Sb) bad_lds[threadIdx.x] = INT_MAX;
  load_rows(lds, stride, gbar, w0, Sb, N, n);
  __syncthreads();
  const int t = threadIdx.x;
  double ga = 0.0, gb = 0.0;
  if (t < 2 * Sb) {
    const int s = t >> 1, p = t & 1;
    double2* x = lds + s * stride;
    double* L1a = reinterpret_cast<double*>(x + NP);
    double* L2a = L1a + NP;
    const double a = ca[w0 + s], b = cb[w0 + s];
    int bad = INT_MAX;
    BihState m2 = {0, 0, 0, 0, 0}, m4 = {0, 0, 0, 0, 0};
    double2 z2 = zero2(), z4 = zero2(), SP = zero2(), SR = zero2();
    Recip R;
    R.init(p);
    for (int k = p; k < n; k += 2) {
      if (k != p) R.advance(k);
      const BihRow h = bih_row(k, a, b, N, gl, R);
      double tm2 = h.hm2, t0 = h.h0, t2 = h.hp2, t4 = h.hp4, P = h.p, Rr = h.r;
      double l1 = 0.0, l2 = 0.0;
      if (k >= 4) {
        l2 = h.hm4 * m4.rU0;
        tm2 = __builtin_fma(-l2, m4.U2, tm2);
        t0 = __builtin_fma(-l2, m4.U4, t0);
        t2 = __builtin_fma(-l2, __builtin_fma(m4.P, h.q2, m4.R * h.s2), t2);
        t4 = __builtin_fma(-l2, __builtin_fma(m4.P, h.q4, m4.R * h.s4), t4);
        P = __builtin_fma(-l2, m4.P, P);
        Rr = __builtin_fma(-l2, m4.R, Rr);
      }
      if (k >= 2) {
        l1 = tm2 * m2.rU0;
        t0 = __builtin_fma(-l1, m2.U2, t0);
        t2 = __builtin_fma(-l1, m2.U4, t2);
        t4 = __builtin_fma(-l1, __builtin_fma(m2.P, h.q4, m2.R * h.s4), t4);
        P = __builtin_fma(-l1, m2.P, P);
        Rr = __builtin_fma(-l1, m2.R, Rr);
      }
      // z_k = (g_k - U2_{k-2} z_{k-2} - U4_{k-4} z_{k-4} - q_k SP - s_k SR) / U0_k
      double2 r = x[k];
      if (k >= 2) r = c_fnms(m2.U2, z2, r);
      if (k >= 4) r = c_fnms(m4.U4, z4, r);
      const double qk = R.p3, sk = ((double)k + 2.0) * ((double)k + 2.0) * R.p3;
      r = c_fnms(qk, SP, r);
      r = c_fnms(sk, SR, r);
      if (bad_pivot(t0, row_scale(h)) && bad == INT_MAX) bad = k;
      const double rU0 = 1.0 / t0;
      const double2 z = c_mul(rU0, r);
      x[k] = z;
      L1a[k] = l1;
      L2a[k] = l2;
      // prefix sums over j <= k-4 for row k+2
      if (k >= 4) {
        SP = c_fma(m4.P, z4, SP);
        SR = c_fma(m4.R, z4, SR);
      }
      m4 = m2;
      z4 = z2;
      m2 = BihState{rU0, t2, t4, P, Rr};
      z2 = z;
    }
    if (bad != INT_MAX) atomicMin(&bad_lds[s], bad);
    const double2* uu = ufwd ? ufwd + (w0 + s) * (int64_t)N : nullptr;
    double2 l2v = zero2(), l4v = zero2();
    int kl = last_of_parity(n, p);
    Recip Rb;
    if (kl >= 0) Rb.init(kl);
    for (int k = kl; k >= 0; k -= 2) {
      if (k != kl) Rb.retreat(k);
      double2 lam = x[k];
      if (k + 2 < n) lam = c_fnms(L1a[k + 2], l2v, lam);
      if (k + 4 < n) lam = c_fnms(L2a[k + 4], l4v, lam);
      x[k] = lam;
      l4v = l2v;
      l2v = lam;
      if (uu != nullptr) {
        const BihMats m = bih_mats(k, N, gl, Rb);
        double2 Au = c_mul(m.A0, uu[k]);
        double2 Bu = c_mul(m.B0, uu[k]);
        if (k >= 2) {
          Au = c_fma(m.Am2, uu[k - 2], Au);
          Bu = c_fma(m.Bm2, uu[k - 2], Bu);
        }
        if (k >= 4) Bu = c_fma(m.Bm4, uu[k - 4], Bu);
        if (k + 2 < n) {
          Au = c_fma(m.A2, uu[k + 2], Au);
          Bu = c_fma(m.B2, uu[k + 2], Bu);
        }
        if (k + 4 < n) Bu = c_fma(m.B4, uu[k + 4], Bu);
        ga -= lam.x * Au.x + lam.y * Au.y;
        gb -= lam.x * Bu.x + lam.y * Bu.y;
      }
    }
  }
  ga += __shfl_xor(ga, 1);
  gb += __shfl_xor(gb, 1);
  if (t < 2 * Sb && (t & 1) == 0 && ufwd != nullptr) {
    if (grad_a) grad_a[w0 + (t >> 1)] = ga;
    if (grad_b) grad_b[w0 + (t >> 1)] = gb;
  }
  __syncthreads();
  store_rows(lam_out, lds, stride, w0, Sb, N, n);
  write_info(info, bad_lds, w0, Sb);
}

// Hu (or H^T u) for the biharmonic matrix.  Layout per system: x double2[NP].
// With rhs != 0 (and trans == 0): ca holds K2 per system and the result is
// the Crank-Nicolson right-hand side sigma S(h) - (Q + a' A + b' B) u, a' =
// inv - 2 K2, b' = K2 (K2 - inv) (sh = S(h) rows, or null).
__global__ __launch_bounds__(kChainThreads) void bih_chain_matvec(int N, int64_t nsys, int S, int NP, const double* __restrict__ ca,
                                                                   const double* __restrict__ cb, const double2* __restrict__ uin,
                                                                   double2* __restrict__ out, int gl, int trans, int rhs, double inv,
                                                                   double sigma, const double2* __restrict__ sh) {
  extern __shared__ double2 lds[];
  const int64_t w0 = (int64_t)blockIdx.x * S;
  const int Sb = (int)min((int64_t)S, nsys - w0);
  const int n = N - 4;
  const int stride = NP;
  load_rows(lds, stride, uin, w0, Sb, N, n);
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 2 * Sb) {
    const int s = t >> 1, p = t & 1;
    const double2* x = lds + s * stride;
    double2* o = out + (w0 + s) * (int64_t)N;
    const double2* so = sh ? sh + (w0 + s) * (int64_t)N : nullptr;
    const double a = rhs ? rhs_a(ca[w0 + s], inv) : ca[w0 + s];
    const double b = rhs ? rhs_b(ca[w0 + s], inv) : cb[w0 + s];
    if (!trans) {
      double2 sq = zero2(), ss = zero2(), u2 = zero2(), u4 = zero2();
      const int kl = last_of_parity(n, p);
      Recip R;
      if (kl >= 0) R.init(kl);
      for (int k = kl; k >= 0; k -= 2) {
        if (k != kl) R.retreat(k);
        const BihRow h = bih_row(k, a, b, N, gl, R);
        const double2 uk = x[k];
        double2 v = c_mul(h.h0, uk);
        v = c_fma(h.hp2, u2, v);
        v = c_fma(h.hp4, u4, v);
        v = c_fma(h.p, sq, v);
        v = c_fma(h.r, ss, v);
        if (k >= 2) v = c_fma(h.hm2, x[k - 2], v);
        if (k >= 4) v = c_fma(h.hm4, x[k - 4], v);
        if (rhs) v = rhs_combine(v, sigma, so ? so + k : nullptr);
        o[k] = v;
        sq = c_fma(h.q4, u4, sq);
        ss = c_fma(h.s4, u4, ss);
        u4 = u2;
        u2 = uk;
      }
    } else {
      // (H^T u)_k = sum_j H_{j,k} u_j: band entries of rows k-4..k+4 at column k,
      // plus q_k sum_{j<=k-6} p_j u_j + s_k sum_{j<=k-6} r_j u_j.
      double2 SPp = zero2(), SRr = zero2();
      double pm2 = 0.0, rm2 = 0.0, pm4 = 0.0, rm4 = 0.0;
      double hp2_m2 = 0.0, hp4_m2 = 0.0, hp4_m4 = 0.0;
      double2 um2 = zero2(), um4 = zero2();
      Recip R;
      R.init(p);
      for (int k = p; k < n; k += 2) {
        if (k != p) R.advance(k);
        const BihRow h = bih_row(k, a, b, N, gl, R);
        const double2 uk = x[k];
        double2 v = c_mul(h.h0, uk);
        if (k >= 2) v = c_fma(hp2_m2, um2, v);
        if (k >= 4) v = c_fma(hp4_m4, um4, v);
        if (k + 2 < n) {
          Recip R2 = R;
          R2.advance(k + 2);
          const BihRow h2 = bih_row(k + 2, a, b, N, gl, R2);
          v = c_fma(h2.hm2, x[k + 2], v);
          if (k + 4 < n) {
            Recip R4 = R2;
            R4.advance(k + 4);
            const BihRow h4 = bih_row(k + 4, a, b, N, gl, R4);
            v = c_fma(h4.hm4, x[k + 4], v);
          }
        }
        const double qk = R.p3, sk = ((double)k + 2.0) * ((double)k + 2.0) * R.p3;
        v = c_fma(qk, SPp, v);
        v = c_fma(sk, SRr, v);
        o[k] = v;
        if (k >= 4) {  // row k+2 needs the sums over j <= k-4
          SPp = c_fma(pm4, um4, SPp);
          SRr = c_fma(rm4, um4, SRr);
        }
        pm4 = pm2;
        rm4 = rm2;
        um4 = um2;
        hp4_m4 = hp4_m2;
        pm2 = h.p;
        rm2 = h.r;
        um2 = uk;
        hp2_m2 = h.hp2;
        hp4_m2 = h.hp4;
      }
    }
  }
  for (int s = 0; s < Sb; ++s)
    for (int k = n + threadIdx.x; k < N; k += kChainThreads) out[(w0 + s) * (int64_t)N + k] = zero2();
}


// ---------------------------------------------------------------------------
// Biharmonic FP32 solve + FP64 refinement.
// Layout per system (bytes): fv double2[NP] | uu double2[NP] | wk float2[NP] |
// fc float[8 NP] (1/U0, U2, U4, P, R, L1, L2, unused).  wk + fc (40 NP bytes)
// hold the 5 NP FP64 factors of the fallback solve.
// ---------------------------------------------------------------------------
struct BihState32 {
  float rU0, U2, U4, P, R;
};

__device__ __forceinline__ void bih_factor32(float* fc, int NP, int p, int n, int N, int gl, double a, double b) {
  BihState32 m2 = {0, 0, 0, 0, 0}, m4 = {0, 0, 0, 0, 0};
  Recip R;
  R.init(p);
  for (int k = p; k < n; k += 2) {
    if (k != p) R.advance(k);
    const BihRow h = bih_row(k, a, b, N, gl, R);
    float tm2 = (float)h.hm2, t0 = (float)h.h0, t2 = (float)h.hp2, t4 = (float)h.hp4, P = (float)h.p, Rr = (float)h.r;
    const float q2 = (float)h.q2, s2 = (float)h.s2, q4 = (float)h.q4, s4 = (float)h.s4;
    float l1 = 0.f, l2 = 0.f;
    if (k >= 4) {
      l2 = (float)h.hm4 * m4.rU0;
      tm2 = __builtin_fmaf(-l2, m4.U2, tm2);
      t0 = __builtin_fmaf(-l2, m4.U4, t0);
      t2 = __builtin_fmaf(-l2, __builtin_fmaf(m4.P, q2, m4.R * s2), t2);
      t4 = __builtin_fmaf(-l2, __builtin_fmaf(m4.P, q4, m4.R * s4), t4);
      P = __builtin_fmaf(-l2, m4.P, P);
      Rr = __builtin_fmaf(-l2, m4.R, Rr);
    }
    if (k >= 2) {
      l1 = tm2 * m2.rU0;
      t0 = __builtin_fmaf(-l1, m2.U2, t0);
      t2 = __builtin_fmaf(-l1, m2.U4, t2);
      t4 = __builtin_fmaf(-l1, __builtin_fmaf(m2.P, q4, m2.R * s4), t4);
      P = __builtin_fmaf(-l1, m2.P, P);
      Rr = __builtin_fmaf(-l1, m2.R, Rr);
    }
    const float rU0 = 1.0f / t0;
    fc[k] = rU0;
    fc[NP + k] = t2;
    fc[2 * NP + k] = t4;
    fc[3 * NP + k] = P;
    fc[4 * NP + k] = Rr;
    fc[5 * NP + k] = l1;
    fc[6 * NP + k] = l2;
    m4 = m2;
    m2 = BihState32{rU0, t2, t4, P, Rr};
  }
}

__device__ __forceinline__ void bih_fwd32(float2* w, const float* fc, int NP, int p, int n) {
  float2 y2 = make_float2(0.f, 0.f), y4 = make_float2(0.f, 0.f);
  for (int k = p; k < n; k += 2) {
    float2 y = w[k];
    if (k >= 4) y = c_fnms(fc[6 * NP + k], y4, y);
    if (k >= 2) y = c_fnms(fc[5 * NP + k], y2, y);
    w[k] = y;
    y4 = y2;
    y2 = y;
  }
}

__device__ __forceinline__ double bih_back32_add(const float2* w, const float* fc, int NP, double2* uu, int p, int n, bool first) {
  float2 d2 = make_float2(0.f, 0.f), d4 = make_float2(0.f, 0.f);
  double2 sq = zero2(), ss = zero2();
  double dmax = 0.0;
  for (int k = last_of_parity(n, p); k >= 0; k -= 2) {
    float2 v = c_fnms(fc[NP + k], d2, w[k]);
    v = c_fnms(fc[2 * NP + k], d4, v);
    v = c_fnms(fc[3 * NP + k], make_float2((float)sq.x, (float)sq.y), v);
    v = c_fnms(fc[4 * NP + k], make_float2((float)ss.x, (float)ss.y), v);
    const float r0 = fc[k];
    const float2 dk = make_float2(r0 * v.x, r0 * v.y);
    const double2 dd = make_double2((double)dk.x, (double)dk.y);
    uu[k] = first ? dd : c_add(uu[k], dd);
    dmax = fmax(dmax, c_abs1(dd));
    const double2 d4d = make_double2((double)d4.x, (double)d4.y);
    sq = c_fma(q_of(k + 4), d4d, sq);
    ss = c_fma(s_of(k + 4), d4d, ss);
    d4 = d2;
    d2 = dk;
  }
  return dmax;
}

// r = f - H u in FP64 (suffix sums of q_j u_j and s_j u_j), stored as complex64.
__device__ __forceinline__ double bih_residual(const double2* fv, const double2* uu, float2* w, int p, int n, int N, int gl, double a,
                                               double b) {
  double2 sq = zero2(), ss = zero2(), u2 = zero2(), u4 = zero2();
  double umax = 0.0;
  const int kl = last_of_parity(n, p);
  Recip R;
  if (kl >= 0) R.init(kl);
  for (int k = kl; k >= 0; k -= 2) {
    if (k != kl) R.retreat(k);
    const BihRow h = bih_row(k, a, b, N, gl, R);
    const double2 uk = uu[k];
    double2 r = c_fnms(h.h0, uk, fv[k]);
    r = c_fnms(h.hp2, u2, r);
    r = c_fnms(h.hp4, u4, r);
    r = c_fnms(h.p, sq, r);
    r = c_fnms(h.r, ss, r);
    if (k >= 2) r = c_fnms(h.hm2, uu[k - 2], r);
    if (k >= 4) r = c_fnms(h.hm4, uu[k - 4], r);
    w[k] = make_float2((float)r.x, (float)r.y);
    umax = fmax(umax, c_abs1(uk));
    sq = c_fma(h.q4, u4, sq);
    ss = c_fma(h.s4, u4, ss);
    u4 = u2;
    u2 = uk;
  }
  return umax;
}

__global__ __launch_bounds__(kChainThreads) void bih_chain_mixed(int N, int64_t nsys, int S, int NP, const double* __restrict__ ca,
                                                                  const double* __restrict__ cb, const double2* __restrict__ f,
                                                                  double2* __restrict__ u, int gl, int32_t* __restrict__ info,
                                                                  int32_t* __restrict__ iters, int it_max, double tol) {
  extern __shared__ double2 lds[];
  const int64_t w0 = (int64_t)blockIdx.x * S;
  const int Sb = (int)min((int64_t)S, nsys - w0);
  const int n = N - 4;
  const int stride = 2 * NP + (40 * NP + 15) / 16;  // double2 units
  int* bad_lds = reinterpret_cast<int*>(lds + (size_t)S * stride);
  if ((int)threadIdx.x < Sb) bad_lds[threadIdx.x] = INT_MAX;
  load_rows(lds, stride, f, w0, Sb, N, n);
  __syncthreads();
  const int t = threadIdx.x;
  const bool act = t < 2 * Sb;
  const int s = t >> 1, p = t & 1;
  double2* fv = lds + s * stride;
  double2* uu = fv + NP;
  float2* wk = reinterpret_cast<float2*>(uu + NP);
  float* fc = reinterpret_cast<float*>(wk + NP);
  const double a = act ? ca[w0 + s] : 0.0, b = act ? cb[w0 + s] : 0.0;
  if (act) {
    for (int k = p; k < n; k += 2) wk[k] = make_float2((float)fv[k].x, (float)fv[k].y);
    bih_factor32(fc, NP, p, n, N, gl, a, b);
    bih_fwd32(wk, fc, NP, p, n);
    bih_back32_add(wk, fc, NP, uu, p, n, true);
  }
  bool running = act, converged = false;
  double prev = 1e300;
  int ncorr = 0;
  if (it_max == 0) {  // the uncorrected FP32 solution, when finite
    running = false;
    const int fin = (act && finite_rows(uu, p, n)) ? 1 : 0;
    converged = act && (fin & __shfl_xor(fin, 1)) != 0;
  }
  for (int it = 1; it <= it_max; ++it) {
    double umax = 0.0, dmax = 0.0;
    if (running) {
      umax = bih_residual(fv, uu, wk, p, n, N, gl, a, b);
      bih_fwd32(wk, fc, NP, p, n);
      dmax = bih_back32_add(wk, fc, NP, uu, p, n, false);
    }
    umax = fmax(umax, __shfl_xor(umax, 1));
    dmax = fmax(dmax, __shfl_xor(dmax, 1));
    if (running) {
      ncorr = it;
      refine_decide(it, it_max, dmax, umax, prev, tol, running, converged);
    }
    if (!__any(running)) break;
  }
  if (act && running) converged = false;
  if (iters != nullptr && act && p == 0) iters[w0 + s] = ncorr;
  if (act && !converged) {
    double2* x = uu;
    double* fac = reinterpret_cast<double*>(wk);
    for (int k = p; k < n; k += 2) x[k] = fv[k];
    const int bad = bih_fwd64(x, fac, NP, p, n, N, gl, a, b);
    if (bad != INT_MAX) atomicMin(&bad_lds[s], bad);
    bih_back64(x, fac, NP, p, n);
    if (bad == INT_MAX) atomicMin(&bad_lds[s], INT_MAX - 1);
  }
  __syncthreads();
  store_rows(u, lds + NP, stride, w0, Sb, N, n);
  __syncthreads();
  if (info != nullptr && (int)threadIdx.x < Sb) {
    const int bb = bad_lds[threadIdx.x];
    info[w0 + threadIdx.x] = (bb == INT_MAX) ? 0 : (bb == INT_MAX - 1 ? -2 : bb + 1);
  }
}

// ===========================================================================
// host-side launchers
// ===========================================================================

static inline int np_of(int N) { return N | 1; }

// bytes of LDS per system for each chain kernel
size_t chain_bytes_per_system(ChainKind kind, int N) {
  const size_t NP = (size_t)np_of(N);
  switch (kind) {
    case ChainKind::HelmSolve: return 32 * NP;
    case ChainKind::HelmAdjoint: return 16 * (NP + (NP + 1) / 2);
    case ChainKind::HelmMatvec: return 16 * NP;
    case ChainKind::HelmMixed: return 48 * NP;
    case ChainKind::BihSolve: return 16 * (NP + (5 * NP + 1) / 2);
    case ChainKind::BihAdjoint: return 32 * NP;
    case ChainKind::BihMatvec: return 16 * NP;
    case ChainKind::BihMixed: return 16 * (2 * NP + (40 * NP + 15) / 16);
  }
  return 0;
}

int chain_systems_per_block(ChainKind kind, int N, size_t lds_budget) {
  const size_t per = chain_bytes_per_system(kind, N) + 4;
  size_t S = lds_budget / per;
  if (S > 32) S = 32;
  return (int)S;
}

hipError_t launch_chain(const ChainArgs& a) {
  const int S = chain_systems_per_block(a.kind, a.N, a.lds_budget);
  if (S < 1) return hipErrorInvalidValue;
  const int NP = np_of(a.N);
  const size_t lds = (size_t)S * chain_bytes_per_system(a.kind, a.N) + 4 * (size_t)S;
  const int64_t blocks = (a.nsys + S - 1) / S;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks), block(kChainThreads);
  hipStream_t st = (hipStream_t)a.stream;
  if (lds > 65536) {
    const void* fn = nullptr;
    switch (a.kind) {
      case ChainKind::HelmSolve: fn = (const void*)helm_chain_solve; break;
      case ChainKind::HelmAdjoint: fn = (const void*)helm_chain_adjoint; break;
      case ChainKind::HelmMatvec: fn = (const void*)helm_chain_matvec; break;
      case ChainKind::HelmMixed: fn = (const void*)helm_chain_mixed; break;
      case ChainKind::BihSolve: fn = (const void*)bih_chain_solve; break;
      case ChainKind::BihAdjoint: fn = (const void*)bih_chain_adjoint; break;
      case ChainKind::BihMatvec: fn = (const void*)bih_chain_matvec; break;
      case ChainKind::BihMixed: fn = (const void*)bih_chain_mixed; break;
    }
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const double2* f = (const double2*)a.f;
  double2* u = (double2*)a.u;
  switch (a.kind) {
    case ChainKind::HelmSolve:
      hipLaunchKernelGGL(helm_chain_solve, grid, block, lds, st, a.N, a.nsys, S, NP, a.c0, f, u, a.gl, a.info);
      break;
    case ChainKind::HelmAdjoint:
      hipLaunchKernelGGL(helm_chain_adjoint, grid, block, lds, st, a.N, a.nsys, S, NP, a.c0, (const double2*)a.ufwd, f, u, a.g0,
                         a.gl, a.info);
      break;
    case ChainKind::HelmMatvec:
      hipLaunchKernelGGL(helm_chain_matvec, grid, block, lds, st, a.N, a.nsys, S, NP, a.c0, f, u, a.gl, a.trans, a.rhs, a.inv,
                         a.sigma, (const double2*)a.sh);
      break;
    case ChainKind::HelmMixed:
      hipLaunchKernelGGL(helm_chain_mixed, grid, block, lds, st, a.N, a.nsys, S, NP, a.c0, f, u, a.gl, a.info, a.iters, a.it_max,
                         a.tol);
      break;
    case ChainKind::BihSolve:
      hipLaunchKernelGGL(bih_chain_solve, grid, block, lds, st, a.N, a.nsys, S, NP, a.c0, a.c1, f, u, a.gl, a.info);
      break;
    case ChainKind::BihAdjoint:
      hipLaunchKernelGGL(bih_chain_adjoint, grid, block, lds, st, a.N, a.nsys, S, NP, a.c0, a.c1, (const double2*)a.ufwd, f, u, a.g0,
                         a.g1, a.gl, a.info);
      break;
    case ChainKind::BihMatvec:
      hipLaunchKernelGGL(bih_chain_matvec, grid, block, lds, st, a.N, a.nsys, S, NP, a.c0, a.c1, f, u, a.gl, a.trans, a.rhs,
                         a.inv, a.sigma, (const double2*)a.sh);
      break;
    case ChainKind::BihMixed:
      hipLaunchKernelGGL(bih_chain_mixed, grid, block, lds, st, a.N, a.nsys, S, NP, a.c0, a.c1, f, u, a.gl, a.info, a.iters,
                         a.it_max, a.tol);
      break;
  }
  return hipGetLastError();
}

}  // namespace shen
