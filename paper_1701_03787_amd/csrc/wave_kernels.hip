// "Wave" kernels: one system spread over 2G lanes of a wavefront, held in
// registers, in a single pass over HBM.
//
// Each odd/even chain of a system (Sec. 4) is cut into G chunks of C
// consecutive chain elements; lane (p, m) owns chunk m of chain p.
//
//  1. A boundary kernel (one lane per chain, no data) runs the exact LU
//     recurrence of the chain and writes, at the start of every chunk, the
//     state the recurrence needs to restart there (Helmholtz: 1/d and g of
//     the previous row; biharmonic: the two previous reduced rows of U).
//     The states are parked in the output row u[w], which the solve
//     overwrites afterwards (so this path needs u != f).
//  2. The solve kernel restarts the factorisation at its chunk start (the
//     same arithmetic as the boundary kernel, so the factors are the ones of
//     the sequential LU), then solves L y = f and U u = y.  Both are affine
//     recurrences; per chunk they are summarised as an affine map (forward:
//     2x2 / scalar transfer, backward: 4x4 / 2x2) and the maps are combined
//     across lanes by a Kogge-Stone scan; each lane then reruns its chunk
//     from the scanned incoming state.
//
// Rows k >= n ("padding" at the end of a chain) get zero factors, which
// makes their maps finite and their contribution exactly zero.
#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>

#include <mutex>
#include <type_traits>
#include <vector>

#include "shen_launch.hpp"
#include "shen_rows.hpp"
#include "shenhip.h"

namespace shen {

// ----------------------------------------------------------------- helpers
template <typename T>
__device__ __forceinline__ T shfl_up_w(T v, int d, int w) {
  return __shfl_up(v, (unsigned)d, w);
}
template <typename T>
__device__ __forceinline__ T shfl_down_w(T v, int d, int w) {
  return __shfl_down(v, (unsigned)d, w);
}
__device__ __forceinline__ double2 shfl_up2(double2 v, int d, int w) {
  return make_double2(__shfl_up(v.x, (unsigned)d, w), __shfl_up(v.y, (unsigned)d, w));
}
__device__ __forceinline__ double2 shfl_down2(double2 v, int d, int w) {
  return make_double2(__shfl_down(v.x, (unsigned)d, w), __shfl_down(v.y, (unsigned)d, w));
}

// DPP row shifts inside a row of 16 lanes with zero fill past the row ends
// (bound_ctrl).  row_shr:D gives lane i the value of lane i-D, row_shl:D the
// value of lane i+D.  A scan partner that does not exist thus arrives as 0,
// and composing with a zero map leaves the running offset unchanged, so the
// Kogge-Stone steps need no lane-dependent selects.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
// The same shift with 1.0 where the source lane does not exist: for the
// diagonal of a map, so that a missing partner composes as the identity
// (G = 32, where a row's own prefix must stay intact for the step that
// joins the two rows of a chain).
template <int CTRL>
__device__ __forceinline__ double dpp_d_one(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0x3FF00000, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int D>
struct RowShift {
  static __device__ __forceinline__ double from_lower(double v) { return dpp_d<0x110 + D>(v); }  // lane i-D
  static __device__ __forceinline__ double from_upper(double v) { return dpp_d<0x100 + D>(v); }  // lane i+D
  static __device__ __forceinline__ double from_lower_one(double v) { return dpp_d_one<0x110 + D>(v); }
  static __device__ __forceinline__ double from_upper_one(double v) { return dpp_d_one<0x100 + D>(v); }
  static __device__ __forceinline__ double2 from_lower(double2 v) { return make_double2(from_lower(v.x), from_lower(v.y)); }
  static __device__ __forceinline__ double2 from_upper(double2 v) { return make_double2(from_upper(v.x), from_upper(v.y)); }
  static __device__ __forceinline__ float from_lower(float v) { return dpp_f<0x110 + D>(v); }
  static __device__ __forceinline__ float from_upper(float v) { return dpp_f<0x100 + D>(v); }
  static __device__ __forceinline__ float2 from_lower(float2 v) { return make_float2(from_lower(v.x), from_lower(v.y)); }
  static __device__ __forceinline__ float2 from_upper(float2 v) { return make_float2(from_upper(v.x), from_upper(v.y)); }
};

// Chains of G = 32 lanes span two DPP rows; the steps that cross from one
// row to the other read single lanes.  Value of lane L of this lane's chain
// (lanes 32p .. 32p + 31 hold the chain of parity p).
template <int L>
__device__ __forceinline__ double chain_lane32(double v, int p) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int lo0 = __builtin_amdgcn_readlane(lo, L), hi0 = __builtin_amdgcn_readlane(hi, L);
  const int lo1 = __builtin_amdgcn_readlane(lo, L + 32), hi1 = __builtin_amdgcn_readlane(hi, L + 32);
  return __hiloint2double(p ? hi1 : hi0, p ? lo1 : lo0);
}
template <int L>
__device__ __forceinline__ double2 chain_lane32(double2 v, int p) {
  return make_double2(chain_lane32<L>(v.x, p), chain_lane32<L>(v.y, p));
}

// FP32 helpers of the mixed-precision form
__device__ __forceinline__ float rcp32(float d) {  // hardware estimate + one Newton step
  const float r = __builtin_amdgcn_rcpf(d);
  return __builtin_fmaf(r, __builtin_fmaf(-d, r, 1.0f), r);
}
__device__ __forceinline__ float2 cf_fma(float s, float2 b, float2 a) {
  return make_float2(__builtin_fmaf(s, b.x, a.x), __builtin_fmaf(s, b.y, a.y));
}
__device__ __forceinline__ float2 cf_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 cf_mul(float s, float2 a) { return make_float2(s * a.x, s * a.y); }
__device__ __forceinline__ float2 to_f2(double2 a) { return make_float2((float)a.x, (float)a.y); }
__device__ __forceinline__ double2 to_d2(float2 a) { return make_double2((double)a.x, (double)a.y); }
__device__ __forceinline__ double cabs1(double2 a) { return fmax(fabs(a.x), fabs(a.y)); }

// Shifts across the G lanes of a chain: value of lane m - D (lo) or m + D
// (hi), zero where that lane does not exist.
template <int G, int D, typename V>
__device__ __forceinline__ V chain_lo(V v, int m) {
  if constexpr (G == 16) {
    return RowShift<D>::from_lower(v);
  } else {
    V o;
    if constexpr (std::is_same_v<V, double2>) {
      o = shfl_up2(v, D, G);
    } else if constexpr (std::is_same_v<V, float2>) {
      o = make_float2(__shfl_up(v.x, (unsigned)D, G), __shfl_up(v.y, (unsigned)D, G));
    } else {
      o = __shfl_up(v, (unsigned)D, G);
    }
    return (m >= D) ? o : V{};
  }
}
template <int G, int D, typename V>
__device__ __forceinline__ V chain_hi(V v, int m) {
  if constexpr (G == 16) {
    return RowShift<D>::from_upper(v);
  } else {
    V o;
    if constexpr (std::is_same_v<V, double2>) {
      o = shfl_down2(v, D, G);
    } else if constexpr (std::is_same_v<V, float2>) {
      o = make_float2(__shfl_down(v.x, (unsigned)D, G), __shfl_down(v.y, (unsigned)D, G));
    } else {
      o = __shfl_down(v, (unsigned)D, G);
    }
    return (m + D < G) ? o : V{};
  }
}



// One Helmholtz LU row step (shared by boundary and solve kernels so that the
// restarted factorisation reproduces the sequential one exactly).
struct HelmPrev {
  double rd, g;  // 1/d and g of row k-2 (ignored for k < 2)
};
__device__ __forceinline__ void helm_step(int k, double al, int N, int gl, const HelmPrev& pv, double& l, double& g, double& rd,
                                          double& d, double& sc) {
  const HelmRow h = helm_row(k, al, N, gl);
  sc = row_scale(h);
  if (k < 2) {
    l = 0.0;
    d = h.h0;
    g = h.hpp;
  } else {
    l = h.hm * pv.rd;
    d = __builtin_fma(-l, pv.g + h.hm, h.h0);
    g = __builtin_fma(-l, pv.g, h.hpp);
  }
  rd = fast_rcp(d);
}
__device__ __forceinline__ void helm_step(int k, double al, int N, int gl, const HelmPrev& pv, double& l, double& g, double& rd,
                                          double& d) {
  double sc;
  helm_step(k, al, N, gl, pv, l, g, rd, d, sc);
}

// The same step in FP32 (mixed-precision form): entries formed in FP64,
// rounded once, factorisation arithmetic in FP32.
struct HelmPrev32 {
  float rd, g;
};
__device__ __forceinline__ void helm_step32(int k, double al, int N, int gl, const HelmPrev32& pv, float& l, float& g, float& rd,
                                            float& d) {
  const HelmRow h = helm_row(k, al, N, gl);
  const float hm = (float)h.hm, h0 = (float)h.h0, hpp = (float)h.hpp;
  if (k < 2) {
    l = 0.0f;
    d = h0;
    g = hpp;
  } else {
    l = hm * pv.rd;
    d = __builtin_fmaf(-l, pv.g + hm, h0);
    g = __builtin_fmaf(-l, pv.g, hpp);
  }
  rd = rcp32(d);
}

// One biharmonic LU row step: row k reduced by rows k-4 (m4) and k-2 (m2).
// Branch-free: for k < 4 (k < 2) the entry hm4 (hm2) is +0 and the state m4
// (m2) is the all-zero state, so the reduction by it adds exact zeros and
// every result is bitwise that of skipping it.
struct BihRowState {
  double rU0, U2, U4, P, R;
};
__device__ __forceinline__ void bih_step_row(const BihRow& h, const BihRowState& m2, const BihRowState& m4, BihRowState& o,
                                             double& l1, double& l2, double& t0out, double& sc) {
  sc = row_scale(h);
  double tm2 = h.hm2, t0 = h.h0, t2 = h.hp2, t4 = h.hp4, P = h.p, Rr = h.r;
  l2 = h.hm4 * m4.rU0;
  tm2 = __builtin_fma(-l2, m4.U2, tm2);
  t0 = __builtin_fma(-l2, m4.U4, t0);
  t2 = __builtin_fma(-l2, __builtin_fma(m4.P, h.q2, m4.R * h.s2), t2);
  t4 = __builtin_fma(-l2, __builtin_fma(m4.P, h.q4, m4.R * h.s4), t4);
  P = __builtin_fma(-l2, m4.P, P);
  Rr = __builtin_fma(-l2, m4.R, Rr);
  l1 = tm2 * m2.rU0;
  t0 = __builtin_fma(-l1, m2.U2, t0);
  t2 = __builtin_fma(-l1, m2.U4, t2);
  t4 = __builtin_fma(-l1, __builtin_fma(m2.P, h.q4, m2.R * h.s4), t4);
  P = __builtin_fma(-l1, m2.P, P);
  Rr = __builtin_fma(-l1, m2.R, Rr);
  o.rU0 = fast_rcp(t0);
  o.U2 = t2;
  o.U4 = t4;
  o.P = P;
  o.R = Rr;
  t0out = t0;
}
__device__ __forceinline__ void bih_step_row(const BihRow& h, const BihRowState& m2, const BihRowState& m4, BihRowState& o,
                                             double& l1, double& l2, double& t0out) {
  double sc;
  bih_step_row(h, m2, m4, o, l1, l2, t0out, sc);
}
__device__ __forceinline__ void bih_step(int k, double a, double b, int N, int gl, const Recip& Rc, const BihRowState& m2,
                                         const BihRowState& m4, BihRowState& o, double& l1, double& l2, double& t0out,
                                         double& sc) {
  bih_step_row(bih_row(k, a, b, N, gl, Rc), m2, m4, o, l1, l2, t0out, sc);
}

// The same step in FP32 (mixed-precision form): row entries formed in FP64
// and rounded once, factorisation arithmetic in FP32.
struct BihRowState32 {
  float rU0, U2, U4, P, R;
};
__device__ __forceinline__ void bih_step_row32(const BihRow& hd, const BihRowState32& m2, const BihRowState32& m4,
                                               BihRowState32& o, float& l1, float& l2, float& t0out) {
  const float hm4 = (float)hd.hm4, hm2 = (float)hd.hm2, h0 = (float)hd.h0, hp2 = (float)hd.hp2, hp4 = (float)hd.hp4;
  const float q2 = (float)hd.q2, s2 = (float)hd.s2, q4 = (float)hd.q4, s4 = (float)hd.s4;
  float tm2 = hm2, t0 = h0, t2 = hp2, t4 = hp4, P = (float)hd.p, Rr = (float)hd.r;
  // branch-free as bih_step_row
  l2 = hm4 * m4.rU0;
  tm2 = __builtin_fmaf(-l2, m4.U2, tm2);
  t0 = __builtin_fmaf(-l2, m4.U4, t0);
  t2 = __builtin_fmaf(-l2, __builtin_fmaf(m4.P, q2, m4.R * s2), t2);
  t4 = __builtin_fmaf(-l2, __builtin_fmaf(m4.P, q4, m4.R * s4), t4);
  P = __builtin_fmaf(-l2, m4.P, P);
  Rr = __builtin_fmaf(-l2, m4.R, Rr);
  l1 = tm2 * m2.rU0;
  t0 = __builtin_fmaf(-l1, m2.U2, t0);
  t2 = __builtin_fmaf(-l1, m2.U4, t2);
  t4 = __builtin_fmaf(-l1, __builtin_fmaf(m2.P, q4, m2.R * s4), t4);
  P = __builtin_fmaf(-l1, m2.P, P);
  Rr = __builtin_fmaf(-l1, m2.R, Rr);
  o.rU0 = rcp32(t0);
  o.U2 = t2;
  o.U4 = t4;
  o.P = P;
  o.R = Rr;
  t0out = t0;
}

// ------------------------------------------------------------------------
// LDS table of BihConst for rows 0 .. RT-1 (RT = 2GC): six 16-byte pairs per
// row, [pair][row'] with row' = k xor ((k / 2C) mod min(2C, 16)).  The rows
// that the lanes of one parity read at one step (one per chunk) then fall in
// distinct 16-byte bank groups, and a row never leaves its chunk's block.
// Pair 0 holds (q4, s4), which the back substitution reads on its own.
// Tables of 1024 rows (G = 32, C = 16) are compact: three pairs, (q4, s4),
// (A0, B0), (B2, B4), the entries that take a division; the polynomial ones
// (bih_poly) are formed on reading, from the same expressions, so both forms
// give the same values.  The full table of 1024 rows and the tiles of four
// wavefronts would exceed the 160 KiB of LDS.
// ------------------------------------------------------------------------
__host__ __device__ constexpr int bih_tab_pairs(int rt) { return rt >= 1024 ? 3 : 6; }
__device__ __forceinline__ int bih_tab_row(int k, int C) {
  const int sh = 31 - __builtin_clz(2 * C);  // log2(2C)
  const int mask = (2 * C - 1) < 15 ? (2 * C - 1) : 15;
  return k ^ ((k >> sh) & mask);
}
// Rows k >= n = N-4 lie outside the system; they are tabulated as identity
// rows (unit diagonal, nothing else), and the couplings of the last rows to
// columns >= n (B2 of rows n-2, n-1 and B4 of rows n-4 .. n-1) are dropped.
// Those entries only ever reach columns >= n, so the factors of the rows
// k < n are unchanged, and a factorisation run on past n yields l = 0 and
// unit pivots there: with a zero right-hand side on those rows the solve
// leaves them exactly zero without any masking.
// TP: table pairs (3 or 6); 0 = bih_tab_pairs(RT).  A kernel that keeps the
// full table at 1024 rows passes 6 to every table routine it calls.
template <int TP = 0>
__device__ __forceinline__ void bih_tab_fill(double* tab, int RT, int C, int N, int gl, int tid, int nthreads) {
  const int pairs = TP ? TP : bih_tab_pairs(RT);
  double2* t2 = reinterpret_cast<double2*>(tab);
  const int n = N - 4;
  for (int k = tid; k < RT; k += nthreads) {
    BihConst c = bih_const(k, N, gl);
    if (k >= n) c = BihConst{0.0, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (k >= n - 2) c.B2 = 0.0;
    if (k >= n - 4) c.B4 = 0.0;
    const int r = bih_tab_row(k, C);
    t2[0 * RT + r] = make_double2(c.q4, c.s4);
    if (pairs == 3) {
      t2[1 * RT + r] = make_double2(c.A0, c.B0);
      t2[2 * RT + r] = make_double2(c.B2, c.B4);
      continue;
    }
    t2[1 * RT + r] = make_double2(c.Am2, c.Q0);
    t2[2 * RT + r] = make_double2(c.A0, c.B0);
    t2[3 * RT + r] = make_double2(c.A2, c.B2);
    t2[4 * RT + r] = make_double2(c.B4, c.p);
    t2[5 * RT + r] = make_double2(c.r, 0.0);
  }
}
template <int TP = 0>
__device__ __forceinline__ BihConst bih_tab_get(const double* tab, int RT, int C, int k) {
  const double2* t2 = reinterpret_cast<const double2*>(tab);
  const int r = bih_tab_row(k, C);
  if ((TP ? TP : bih_tab_pairs(RT)) == 3) {
    // compact table: A0 is nonzero on every row of the system and zero on the
    // identity rows past it, which take Q0 = 1 and no other entry
    const double2 v0 = t2[0 * RT + r], v1 = t2[1 * RT + r], v2 = t2[2 * RT + r];
    const bool real = v1.x != 0.0;
    const BihPoly q = bih_poly(k);
    BihConst c;
    c.q4 = v0.x;
    c.s4 = v0.y;
    c.A0 = v1.x;
    c.B0 = v1.y;
    c.B2 = v2.x;
    c.B4 = v2.y;
    c.Am2 = real ? q.Am2 : 0.0;
    c.Q0 = real ? q.Q0 : 1.0;
    c.A2 = real ? q.A2 : 0.0;
    c.p = real ? q.p : 0.0;
    c.r = real ? q.r : 0.0;
    return c;
  }
  const double2 v0 = t2[0 * RT + r], v1 = t2[1 * RT + r], v2 = t2[2 * RT + r], v3 = t2[3 * RT + r], v4 = t2[4 * RT + r],
                v5 = t2[5 * RT + r];
  BihConst c;
  c.q4 = v0.x;
  c.s4 = v0.y;
  c.Am2 = v1.x;
  c.Q0 = v1.y;
  c.A0 = v2.x;
  c.B0 = v2.y;
  c.A2 = v3.x;
  c.B2 = v3.y;
  c.B4 = v4.x;
  c.p = v4.y;
  c.r = v5.x;
  return c;
}
// (q_{k+4}, s_{k+4}) of row k
__device__ __forceinline__ double2 bih_tab_qs(const double* tab, int C, int k) {
  return reinterpret_cast<const double2*>(tab)[bih_tab_row(k, C)];
}
// constants of a row k >= -4: from the table for k >= 0; for k < 0 only
// q4, s4 (= q_{k+4}, s_{k+4}) exist, everything else is +0, so that the
// entries below the diagonal of rows 0 .. 3 assemble to +0 unmasked
// (field-wise selects rather than a branch: a branch between two whole
// structs is kept in scratch memory)
template <int TP = 0>
__device__ __forceinline__ BihConst bih_const_at(const double* tab, int RT, int C, int k, int N, int gl) {
  const bool neg = k < 0;
  BihConst c = bih_tab_get<TP>(tab, RT, C, neg ? 0 : k);
  const double K = (double)k;
  const double p7 = fast_rcp(K + 7.0);
  const double q4n = p7, s4n = (K + 6.0) * (K + 6.0) * p7;  // as bih_const
  c.Am2 = neg ? 0.0 : c.Am2;
  c.Q0 = neg ? 0.0 : c.Q0;
  c.A0 = neg ? 0.0 : c.A0;
  c.B0 = neg ? 0.0 : c.B0;
  c.A2 = neg ? 0.0 : c.A2;
  c.B2 = neg ? 0.0 : c.B2;
  c.B4 = neg ? 0.0 : c.B4;
  c.p = neg ? 0.0 : c.p;
  c.r = neg ? 0.0 : c.r;
  c.q4 = neg ? q4n : c.q4;
  c.s4 = neg ? s4n : c.s4;
  (void)N;
  (void)gl;
  return c;
}

// =========================================================================
// Boundary kernels: one thread per chain.
// =========================================================================

// States parked in u[w] (as doubles): Helmholtz [(p*G + m)*2 + {0,1}] = (1/d, g)
// of row 2(mC)-2+p; biharmonic [(p*G + m)*10 + ...] = rows k-2 then k-4.
// FP32 restart states (float2 (1/d, g) at float2 slot p*G + m of u[w]).
__global__ __launch_bounds__(256) void helm_boundary32(int N, int64_t nsys, int C, int G, const double* __restrict__ alpha,
                                                       double2* __restrict__ u, int gl) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * nsys) return;
  const int64_t w = t >> 1;
  const int p = (int)(t & 1);
  const int n = N - 2;
  const int nc = (n - p + 1) / 2;
  const int nchunks = (nc + C - 1) / C;
  if (nchunks <= 1) return;
  const double al = alpha[w];
  float2* st = reinterpret_cast<float2*>(u + w * (int64_t)N);
  HelmPrev32 pv = {0.0f, 0.0f};
  const int ilast = (nchunks - 1) * C;
  for (int i = 0; i < ilast; ++i) {
    float l, g, rd, d;
    helm_step32(2 * i + p, al, N, gl, pv, l, g, rd, d);
    pv.rd = rd;
    pv.g = g;
    if ((i + 1) % C == 0) st[p * G + (i + 1) / C] = make_float2(pv.rd, pv.g);
  }
}

// The same walk with the chunk geometry fixed at compile time: the restart
// states are kept in registers and written at the end.  For G <= 16 they go
// out through LDS, one parity at a time, so that every store instruction
// writes whole 256-byte runs of consecutive slots (4 systems x G slots)
// instead of 16-byte pieces of 64 different lines.
// Block blk of the walk over one grid's systems (256 threads, 128 systems).
template <int C, int G>
__device__ __forceinline__ void helm_walk_block(int N, int64_t nsys, const double* __restrict__ alpha,
                                                double2* __restrict__ S, int64_t sstride, int gl, int64_t blk) {
  const int64_t t = blk * 256 + threadIdx.x;
  const bool act = t < 2 * nsys;
  if constexpr (G > 16) {
    if (!act) return;
  }
  const int64_t w = act ? t >> 1 : 0;
  const int p = (int)(t & 1);
  const int n = N - 2;
  const int nc = (n - p + 1) / 2;
  const int nchunks = (nc + C - 1) / C;
  const double al = alpha[w];
  double2 st[G];
  st[0] = zero2();
  HelmPrev pv = {0.0, 0.0};
#pragma unroll
  for (int mm = 1; mm < G; ++mm) {
    st[mm] = zero2();
    if (mm < nchunks) {
#pragma unroll
      for (int j = 0; j < C; ++j) {
        double l, g, rd, d;
        helm_step(2 * ((mm - 1) * C + j) + p, al, N, gl, pv, l, g, rd, d);
        pv.rd = rd;
        pv.g = g;
      }
      st[mm] = make_double2(pv.rd, pv.g);
    }
  }
  if constexpr (G > 16) {
    double2* dst = S + w * sstride + p * G;  // states at (p G + m) of the system's slot, 16 bytes each
#pragma unroll
    for (int mm = 1; mm < G; ++mm)
      if (mm < nchunks) dst[mm] = st[mm];
  } else {
    // wavefront wv holds systems w0 .. w0+31, lane l system w0 + l/2, parity l&1
    __shared__ double2 stage[4][32 * G];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t w0 = (blk * 256 + wv * 64) >> 1;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (p == h) {
#pragma unroll
        for (int mm = 0; mm < G; ++mm) stage[wv][(lane >> 1) * G + mm] = st[mm];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int r = 0; r < G / 2; ++r) {
        const int idx = r * 64 + lane;
        const int64_t ws = w0 + idx / G;
        if (ws < nsys) S[ws * sstride + h * G + idx % G] = stage[wv][idx];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
}

template <int C, int G>
__global__ __launch_bounds__(256) void helm_boundary_t(int N, int64_t nsys, const double* __restrict__ alpha,
                                                       double2* __restrict__ S, int64_t sstride, int gl) {
  helm_walk_block<C, G>(N, nsys, alpha, S, sstride, gl, blockIdx.x);
}

// Table-driven form of the biharmonic boundary walk: the rows are assembled
// from the LDS table (bih_row_tab), exactly as the table-driven wave solves
// assemble them, so the restart states continue the same factorisation.
// States of chunk m go to st[(p G + m) 10 + 0..9] (FP64, or FP32 with F32).
// Each wavefront of a block walks chains of one parity, so every step reads
// one table row for the whole wavefront (broadcast).
// The FP64 walk (F32 false) also checks every pivot of the chain, the last
// chunk's included, with the wave solves' rule, and leaves the first unusable
// row (or -1) in the unused state slot of chunk 0, so that the wave solves
// need not check their rows again.  CHECK false (a one-call solve without
// info): no checks, and no steps past the last chunk start.
template <int C, int G, bool F32, int TP = 0, bool CHECK = !F32>
__device__ __forceinline__ void bih_walk_tab(int N, int p, double a, double b, void* st, int gl, const double* tab) {
  constexpr int RT = 2 * G * C;
  const int n = N - 4;
  const int nc = (n - p + 1) / 2;
  const int nchunks = (nc + C - 1) / C;
  if (F32 && nchunks <= 1) return;
  // only the constants of rows k-2 (B2, q4, s4) and k-4 (B4) are carried
  const BihConst c2 = bih_const_at<TP>(tab, RT, C, p - 2, N, gl), c4 = bih_const_at<TP>(tab, RT, C, p - 4, N, gl);
  double B2m2 = c2.B2, q4m2 = c2.q4, s4m2 = c2.s4, B4m2 = c2.B4, B4m4 = c4.B4;
  using State = typename std::conditional<F32, BihRowState32, BihRowState>::type;
  State m2 = {0, 0, 0, 0, 0}, m4 = {0, 0, 0, 0, 0};
  int bad = INT_MAX;
  auto row = [&](int i) {
    const int k = 2 * i + p;
    const BihConst c = bih_tab_get<TP>(tab, RT, C, k);
    const BihRow h = bih_row_tab(k, a, b, c, B2m2, q4m2, s4m2, B4m4);
    State o;
    if constexpr (F32) {
      float l1, l2, t0;
      bih_step_row32(h, m2, m4, o, l1, l2, t0);
    } else {
      double l1, l2, t0, sc;
      bih_step_row(h, m2, m4, o, l1, l2, t0, sc);
      if constexpr (CHECK) bad = first_bad(bad, i < nc && bad_pivot(t0, sc), k);
    }
    m4 = m2;
    m2 = o;
    B4m4 = B4m2;
    B4m2 = c.B4;
    B2m2 = c.B2;
    q4m2 = c.q4;
    s4m2 = c.s4;
  };
  // one chunk of rows per iteration (unrolled, so the carried state is
  // renamed rather than copied), then the restart state of the next chunk
  for (int mm = 1; mm < nchunks; ++mm) {
#pragma unroll
    for (int j = 0; j < C; ++j) row((mm - 1) * C + j);
    if constexpr (F32) {
      float2* sv = reinterpret_cast<float2*>(reinterpret_cast<float*>(st) + (p * G + mm) * 10);
      sv[0] = make_float2(m2.rU0, m2.U2);
      sv[1] = make_float2(m2.U4, m2.P);
      sv[2] = make_float2(m2.R, m4.rU0);
      sv[3] = make_float2(m4.U2, m4.U4);
      sv[4] = make_float2(m4.P, m4.R);
    } else {
      double2* sv = reinterpret_cast<double2*>(reinterpret_cast<double*>(st) + (p * G + mm) * 10);
      sv[0] = make_double2(m2.rU0, m2.U2);
      sv[1] = make_double2(m2.U4, m2.P);
      sv[2] = make_double2(m2.R, m4.rU0);
      sv[3] = make_double2(m4.U2, m4.U4);
      sv[4] = make_double2(m4.P, m4.R);
    }
  }
  if constexpr (!F32 && CHECK) {
    const int i0 = (nchunks > 1 ? nchunks - 1 : 0) * C;
    for (int i = i0; i < nc; ++i) row(i);
    double2* sv = reinterpret_cast<double2*>(reinterpret_cast<double*>(st) + (p * G) * 10);
    sv[0] = make_double2(bad == INT_MAX ? -1.0 : (double)bad, 0.0);
  }
}

// First unusable row of chain lane (m == 0) from the walk's slot of chunk 0
// (INT_MAX: none, or not a chunk-0 lane).
__device__ __forceinline__ int walk_bad_of(double v, bool chunk0) { return (chunk0 && v >= 0.0) ? (int)v : INT_MAX; }

// Six wavefronts (three pairs of parities, 192 systems) share one table.  At
// most three tables fit a CU, so every block of a channel-size launch is
// resident at once; six-wavefront blocks spread the wavefronts over the SIMDs
// more evenly (at most five per SIMD at 131,584 systems, where eight-wavefront
// blocks leave six on the CUs that take a third block).
static constexpr int kBihWalkThreads = 384;
static constexpr int kBihWalkSystems = kBihWalkThreads / 2;
template <int C, int G, bool F32, bool CHECK = !F32>
__global__ __launch_bounds__(kBihWalkThreads) void bih_boundary_tab(int N, int64_t nsys, const double* __restrict__ ca,
                                                                    const double* __restrict__ cb, double2* __restrict__ S,
                                                                    int64_t sstride, int gl) {
  extern __shared__ double tab[];
  // the FP32 walk serves the FP32 + refinement kernel, which keeps the full table
  constexpr int TP = F32 ? 6 : 0;
  bih_tab_fill<TP>(tab, 2 * G * C, C, N, gl, threadIdx.x, kBihWalkThreads);
  __syncthreads();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * kBihWalkSystems + (wv >> 1) * 64 + lane;
  if (w >= nsys) return;
  bih_walk_tab<C, G, F32, TP, CHECK>(N, wv & 1, ca[w], cb[w], S + w * sstride, gl, tab);
}

// =========================================================================
// Chains longer than one wavefront (large N).  A work group of W wavefronts
// holds one system; wavefront v owns chain elements v*G*C .. (v+1)*G*C - 1 of
// both parity chains (its lanes laid out as in the one-wavefront case).  Each
// scan of the wave solves runs inside every wavefront as before; the
// wavefronts then publish their totals in LDS and each folds the totals of
// the wavefronts before it (forward scans) or after it (backward scan) into
// the state entering its own segment.  A lane's incoming state is then its
// neighbour's inclusive map applied to that state.
// =========================================================================
struct NoCarry {
  static constexpr bool on = false;
  __device__ __forceinline__ int parity(int h) const { return h; }
  __device__ __forceinline__ int kbase(int, int, int) const { return 0; }
};
static constexpr int kCarryMaxW = 4;     // wavefronts per work group
static constexpr int kCarryWords = 24;   // doubles per (scan, segment)
// Publish this segment's map (`owner` lane: the one holding the segment's
// total), wait for the work group, then fold the maps of the segments before
// this one (forward) or after it, from the top down (backward):
// s <- M_u s + c_u, from s = 0.  Segment u's slot is base + u * stride.
template <int D, bool BWD>
__device__ __forceinline__ void fold_segments(double* base, int stride, int seg, int nseg, bool owner,
                                              const double (&M)[D][D], const double2 (&c)[D], double2 (&st)[D]) {
  if (owner) {
    double* o = base + seg * stride;
#pragma unroll
    for (int r = 0; r < D; ++r) {
#pragma unroll
      for (int q = 0; q < D; ++q) o[r * D + q] = M[r][q];
      o[D * D + 2 * r] = c[r].x;
      o[D * D + 2 * r + 1] = c[r].y;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < D; ++r) st[r] = zero2();
  const int cnt = BWD ? nseg - 1 - seg : seg;
  for (int i = 0; i < cnt; ++i) {
    const int u = BWD ? nseg - 1 - i : i;
    const double* o = base + u * stride;
    double2 ns[D];
#pragma unroll
    for (int r = 0; r < D; ++r) {
      double2 acc = make_double2(o[D * D + 2 * r], o[D * D + 2 * r + 1]);
#pragma unroll
      for (int q = 0; q < D; ++q) acc = c_fma(o[r * D + q], st[q], acc);
      ns[r] = acc;
    }
#pragma unroll
    for (int r = 0; r < D; ++r) st[r] = ns[r];
  }
}
// Both parity chains of one system per work group: wavefront v holds segment
// v of each (its lower G lanes parity 0, its upper G lanes parity 1).
struct WaveCarry {
  static constexpr bool on = true;
  int v, W;     // this wavefront, wavefronts per system
  double* xch;  // LDS: [3 scans][kCarryMaxW][2 parities][kCarryWords]
  __device__ __forceinline__ int parity(int h) const { return h; }
  // first row of this wavefront's chain segments (chunk length C, G lanes)
  __device__ __forceinline__ int kbase(int C, int G, int) const { return 2 * v * G * C; }
  template <int D, bool BWD>
  __device__ __forceinline__ void fold(int scan, int h, bool owner, const double (&M)[D][D], const double2 (&c)[D],
                                       double2 (&st)[D]) const {
    fold_segments<D, BWD>(xch + ((scan * kCarryMaxW) * 2 + h) * kCarryWords, 2 * kCarryWords, v, W, owner, M, c, st);
  }
};
// One parity chain per work group (N past what two-parity work groups hold):
// the 2W half-wavefronts of G lanes are consecutive segments of that chain,
// half h of wavefront v being segment 2v + h.
struct ChainCarry {
  static constexpr bool on = true;
  int v, W, pp;  // this wavefront, wavefronts per chain, the chain's parity
  double* xch;   // LDS: [3 scans][2 kCarryMaxW segments][kCarryWords]
  __device__ __forceinline__ int parity(int) const { return pp; }
  __device__ __forceinline__ int kbase(int C, int G, int h) const { return 2 * (2 * v + h) * G * C; }
  template <int D, bool BWD>
  __device__ __forceinline__ void fold(int scan, int h, bool owner, const double (&M)[D][D], const double2 (&c)[D],
                                       double2 (&st)[D]) const {
    fold_segments<D, BWD>(xch + scan * 2 * kCarryMaxW * kCarryWords, kCarryWords, 2 * v + h, 2 * W, owner, M, c, st);
  }
};

// =========================================================================
// Helmholtz wave solve
// =========================================================================
// Solves systems wbase + (lane / 2G) of the wavefront (those below nsys).
template <int C, int G, bool PIPE = false, typename Carry = NoCarry>
__device__ __forceinline__ int helm_wave_core(int N, int lane, int64_t w, bool wok, double al, HelmPrev pv, double2 (&x)[C],
                                              double2* __restrict__ urow, int gl, int32_t* __restrict__ info,
                                              Carry cy = Carry());

template <int C, int G>
__device__ __forceinline__ void helm_wave_body(int N, int64_t nsys, int64_t wbase, const double* __restrict__ alpha,
                                               const double2* __restrict__ f, double2* __restrict__ u,
                                               const double2* __restrict__ sts, int64_t sstride, int gl,
                                               int32_t* __restrict__ info) {
  // opaque lane index: when this body sits in a loop (batched kernels), the
  // per-row constants derived from it are not hoisted out and held across it
  int lane = threadIdx.x & 63;
  asm volatile("" : "+v"(lane));
  lane &= 63;  // opaque, but known to be a lane index
  const int sl = lane / (2 * G);
  const int p = (lane / G) & 1;
  const int m = lane % G;
  const int64_t w = wbase + sl;
  const bool wok = w < nsys;
  const int n = N - 2;
  const int k0 = 2 * m * C + p;
  const double al = wok ? alpha[w] : 0.0;
  const double2* frow = f + (wok ? w : 0) * (int64_t)N;
  double2* urow = u + (wok ? w : 0) * (int64_t)N;

  // restart state of the LU at the chunk start
  HelmPrev pv = {0.0, 0.0};
  if (wok && m > 0 && k0 < n) {
    const double2 s = sts[w * sstride + p * G + m];
    pv.rd = s.x;
    pv.g = s.y;
  }
  double2 x[C];
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int k = k0 + 2 * j;
    x[j] = (wok && k < n) ? frow[k] : zero2();
  }
  helm_wave_core<C, G>(N, lane, w, wok, al, pv, x, urow, gl, info);
}

// Everything after the loads: x holds f of this lane's chunk (0 where k >= n),
// pv the restart state.  Without PIPE the solution is stored to urow; with
// PIPE it is left in x for the caller.
template <int C, int G, bool PIPE, typename Carry>
__device__ __forceinline__ int helm_wave_core(int N, int lane, int64_t w, bool wok, double al, HelmPrev pv, double2 (&x)[C],
                                              double2* __restrict__ urow, int gl, int32_t* __restrict__ info, Carry cy) {
  const int hf = (lane / G) & 1;  // which G-lane half of the 2G lanes
  const int p = cy.parity(hf);    // the parity of this lane's chain
  const int m = lane % G;
  const int n = N - 2;
  const int k0 = cy.kbase(C, G, hf) + 2 * m * C + p;
  const double hm = -0.5 * kPi * al;
  // factorisation restart + local forward elimination (zero incoming state)
  // l of row k is hm times 1/d of row k-2 (helm_step), so it is rebuilt from
  // rdj where needed instead of being kept.
  double rdj[C], gj[C];
  const double rd_in = (k0 >= 2) ? pv.rd : 0.0;
  int bad = INT_MAX;
  double T = 1.0;
  double2 yp = zero2();
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int k = k0 + 2 * j;
    const bool ok = wok && k < n;
    double l, g, rd, d, sc;
    helm_step(k, al, N, gl, pv, l, g, rd, d, sc);
    bad = first_bad(bad, ok && bad_pivot(d, sc), k);
    pv.rd = rd;
    pv.g = g;
    l = ok ? l : 0.0;
    rdj[j] = ok ? rd : 0.0;
    gj[j] = ok ? g : 0.0;
    const double2 y = c_fnms(l, yp, x[j]);
    x[j] = y;
    yp = y;
    T *= -l;
  }
  // forward scan over chunks: (T, b) with b = last y; compose(later, earlier)
  double sT = T;
  double2 sb = yp;
  double2 h;
  if constexpr (G == 16 && !Carry::on) {
    auto lvl = [&](auto sh) {
      using S = decltype(sh);
      const double oT = S::from_lower(sT);
      const double2 ob = S::from_lower(sb);
      sb = c_fma(sT, ob, sb);
      sT = sT * oT;
    };
    lvl(RowShift<1>{});
    lvl(RowShift<2>{});
    lvl(RowShift<4>{});
    lvl(RowShift<8>{});
    h = RowShift<1>::from_lower(sb);
  } else {
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
      const double oT = shfl_up_w(sT, d, G);
      const double2 ob = shfl_up2(sb, d, G);
      if (m >= d) {
        sb = c_fma(sT, ob, sb);
        sT = sT * oT;
      }
    }
    if constexpr (Carry::on) {
      // y entering this wavefront's segment, then entering this lane
      const double M[1][1] = {{sT}};
      const double2 c[1] = {sb};
      double2 sin[1];
      cy.template fold<1, false>(0, hf, m == G - 1, M, c, sin);
      h = c_sel(m == 0, sin[0], shfl_up2(c_fma(sT, sin[0], sb), 1, G));
    } else {
      h = shfl_up2(sb, 1, G);
      if (m == 0) h = zero2();
    }
  }
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const bool ok = wok && k0 + 2 * j < n;
    const double l = ok ? hm * (j == 0 ? rd_in : rdj[j - 1]) : 0.0;
    h = c_mul(-l, h);
    x[j] = c_add(x[j], h);
  }
  // backward: state (a = u_{i+1}, S = S_{i+2});  u_i = yh - eh a - gh S
  double eh[C], gh[C];
  double A00 = 1.0, A01 = 0.0, A10 = 0.0, A11 = 1.0;
  double2 c0 = zero2(), c1 = zero2();
#pragma unroll
  for (int j = C - 1; j >= 0; --j) {
    const double r = rdj[j];
    x[j] = c_mul(r, x[j]);  // yh
    eh[j] = (r == 0.0) ? 0.0 : r * (gj[j] + hm);
    gh[j] = r * gj[j];
    // M = [[-eh, -gh], [1, 1]];  A <- M A ; c <- M c + (yh, 0)
    const double n00 = -eh[j] * A00 - gh[j] * A10, n01 = -eh[j] * A01 - gh[j] * A11;
    const double n10 = A00 + A10, n11 = A01 + A11;
    A00 = n00;
    A01 = n01;
    A10 = n10;
    A11 = n11;
    double2 nc0 = c_fma(-eh[j], c0, x[j]);
    nc0 = c_fma(-gh[j], c1, nc0);
    const double2 nc1 = c_add(c0, c1);
    c0 = nc0;
    c1 = nc1;
  }
  // suffix scan: compose(lower, higher) = (A_lo A_hi, A_lo c_hi + c_lo)
  auto compose2 = [&](double o00, double o01, double o10, double o11, double2 oc0, double2 oc1) {
    const double2 n0 = c_add(c_fma(A00, oc0, c_mul(A01, oc1)), c0);
    const double2 n1 = c_add(c_fma(A10, oc0, c_mul(A11, oc1)), c1);
    const double n00 = A00 * o00 + A01 * o10, n01 = A00 * o01 + A01 * o11;
    const double n10 = A10 * o00 + A11 * o10, n11 = A10 * o01 + A11 * o11;
    A00 = n00;
    A01 = n01;
    A10 = n10;
    A11 = n11;
    c0 = n0;
    c1 = n1;
  };
  double2 sa, sS;
  if constexpr (G == 16 && !Carry::on) {
    auto lvl = [&](auto sh) {
      using S = decltype(sh);
      compose2(S::from_upper(A00), S::from_upper(A01), S::from_upper(A10), S::from_upper(A11), S::from_upper(c0),
               S::from_upper(c1));
    };
    lvl(RowShift<1>{});
    lvl(RowShift<2>{});
    lvl(RowShift<4>{});
    lvl(RowShift<8>{});
    sa = RowShift<1>::from_upper(c0);
    sS = RowShift<1>::from_upper(c1);
  } else {
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
      const double o00 = shfl_down_w(A00, d, G), o01 = shfl_down_w(A01, d, G);
      const double o10 = shfl_down_w(A10, d, G), o11 = shfl_down_w(A11, d, G);
      const double2 oc0 = shfl_down2(c0, d, G), oc1 = shfl_down2(c1, d, G);
      if (m + d < G) compose2(o00, o01, o10, o11, oc0, oc1);
    }
    if constexpr (Carry::on) {
      // state entering this wavefront's segment from above, then this lane
      const double M[2][2] = {{A00, A01}, {A10, A11}};
      const double2 c[2] = {c0, c1};
      double2 top[2];
      cy.template fold<2, true>(1, hf, m == 0, M, c, top);
      sa = c_sel(m == G - 1, top[0], shfl_down2(c_add(c_fma(A00, top[0], c_mul(A01, top[1])), c0), 1, G));
      sS = c_sel(m == G - 1, top[1], shfl_down2(c_add(c_fma(A10, top[0], c_mul(A11, top[1])), c1), 1, G));
    } else {
      sa = shfl_down2(c0, 1, G);
      sS = shfl_down2(c1, 1, G);
      if (m == G - 1) {
        sa = zero2();
        sS = zero2();
      }
    }
  }
#pragma unroll
  for (int j = C - 1; j >= 0; --j) {
    double2 uj = c_fma(-eh[j], sa, x[j]);
    uj = c_fma(-gh[j], sS, uj);
    x[j] = uj;
    sS = c_add(sS, sa);
    sa = uj;
  }
  if constexpr (!PIPE) {
    if (wok) {
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const int k = k0 + 2 * j;
        if (k < N) urow[k] = (k < n) ? x[j] : zero2();
      }
    }
  }
  if (info != nullptr) {
    // min over the 2G lanes of the system
    int b = bad;
#pragma unroll
    for (int d = 1; d < 2 * G; d <<= 1) b = min(b, __shfl_xor(b, d, 2 * G));
    if (wok && (lane % (2 * G)) == 0) info[w] = (b == INT_MAX) ? 0 : b + 1;
  }
  return bad;
}

// =========================================================================
// Helmholtz adjoint (wave layout): lambda = H^{-T} gbar and, when asked,
// grad_alpha = -Re(lambda^H B u).  H^T = U^T L^T: U^T z = gbar runs forward
// with the state (z of row k-2, sum of g_i z_i over rows <= k-4), an affine
// 2x2 recurrence scanned like the forward solve's; L^T lambda = z runs
// backward, scalar.  Restart states come from the same boundary walk as the
// solve (parked in the lambda row, so lambda must not alias gbar).
// =========================================================================
template <int C, int G>
__global__ __launch_bounds__(64) void helm_adjoint_wave(int N, int64_t nsys, const double* __restrict__ alpha,
                                                        const double2* __restrict__ ufwd, const double2* __restrict__ gbar,
                                                        double2* __restrict__ lam, const double2* __restrict__ sts,
                                                        int64_t sstride, double* __restrict__ grad, int gl,
                                                        int32_t* __restrict__ info) {
  constexpr int SPW = 64 / (2 * G);
  const int lane = threadIdx.x & 63;
  const int sl = lane / (2 * G), p = (lane / G) & 1, m = lane % G;
  const int64_t w = (int64_t)blockIdx.x * SPW + sl;
  const bool wok = w < nsys;
  const int n = N - 2;
  const int k0 = 2 * m * C + p;
  const double al = wok ? alpha[w] : 0.0;
  const double hm = -0.5 * kPi * al;
  const double2* grow = gbar + (wok ? w : 0) * (int64_t)N;
  double2* lrow = lam + (wok ? w : 0) * (int64_t)N;
  HelmPrev pv = {0.0, 0.0};
  if (wok && m > 0 && k0 < n) {
    const double2 s2 = sts[w * sstride + p * G + m];
    pv.rd = s2.x;
    pv.g = s2.y;
  }
  double2 x[C];
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int k = k0 + 2 * j;
    x[j] = (wok && k < n) ? grow[k] : zero2();
  }
  // factorisation restart (as the solve)
  const bool has_prev = k0 >= 2;
  const double g_in = has_prev ? pv.g : 0.0;
  double rdj[C], gj[C];
  int bad = INT_MAX;
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int k = k0 + 2 * j;
    const bool ok = wok && k < n;
    double l, g, r, d, sc;
    helm_step(k, al, N, gl, pv, l, g, r, d, sc);
    bad = first_bad(bad, ok && bad_pivot(d, sc), k);
    pv.rd = r;
    pv.g = g;
    rdj[j] = ok ? r : 0.0;
    gj[j] = ok ? g : 0.0;
  }
  // U^T z = gbar: local pass from a zero state, composing the chunk's map
  // state (zp, P) -> (z_j, P + g_{j-1} zp);  z_j = rd_j (gbar_j - e_{j-1} zp - P)
  auto gprev = [&](int j) { return j == 0 ? g_in : gj[j == 0 ? 0 : j - 1]; };
  auto eprev = [&](int j) {
    const double g = gprev(j);
    return (j == 0 && !has_prev) ? 0.0 : g + hm;
  };
  double A00 = 1.0, A01 = 0.0, A10 = 0.0, A11 = 1.0;
  double2 c0 = zero2(), c1 = zero2();
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const double r = rdj[j], e = eprev(j), g = gprev(j);
    // M = [[-r e, -r], [g, 1]]
    const double m00 = -r * e, m01 = -r;
    const double n00 = m00 * A00 + m01 * A10, n01 = m00 * A01 + m01 * A11;
    const double n10 = g * A00 + A10, n11 = g * A01 + A11;
    A00 = n00;
    A01 = n01;
    A10 = n10;
    A11 = n11;
    double2 z = c_mul(r, x[j]);
    z = c_fma(m00, c0, z);
    z = c_fma(m01, c1, z);
    const double2 nP = c_fma(g, c0, c1);
    c0 = z;
    c1 = nP;
  }
  auto compose = [&](double o00, double o01, double o10, double o11, double2 oc0, double2 oc1) {
    // (this after other): (A A_o, A c_o + c)
    const double2 n0 = c_add(c_fma(A00, oc0, c_mul(A01, oc1)), c0);
    const double2 n1 = c_add(c_fma(A10, oc0, c_mul(A11, oc1)), c1);
    const double n00 = A00 * o00 + A01 * o10, n01 = A00 * o01 + A01 * o11;
    const double n10 = A10 * o00 + A11 * o10, n11 = A10 * o01 + A11 * o11;
    A00 = n00;
    A01 = n01;
    A10 = n10;
    A11 = n11;
    c0 = n0;
    c1 = n1;
  };
  auto lvl = [&](auto dd) {
    constexpr int D = decltype(dd)::value;
    compose(chain_lo<G, D>(A00, m), chain_lo<G, D>(A01, m), chain_lo<G, D>(A10, m), chain_lo<G, D>(A11, m),
            chain_lo<G, D>(c0, m), chain_lo<G, D>(c1, m));
  };
  lvl(std::integral_constant<int, 1>{});
  if constexpr (G > 2) lvl(std::integral_constant<int, 2>{});
  if constexpr (G > 4) lvl(std::integral_constant<int, 4>{});
  if constexpr (G > 8) lvl(std::integral_constant<int, 8>{});
  if constexpr (G > 16) lvl(std::integral_constant<int, 16>{});
  double2 zp = chain_lo<G, 1>(c0, m), P = chain_lo<G, 1>(c1, m);
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const double r = rdj[j], e = eprev(j), g = gprev(j);
    double2 z = c_mul(r, x[j]);
    z = c_fma(-r * e, zp, z);
    z = c_fma(-r, P, z);
    P = c_fma(g, zp, P);
    zp = z;
    x[j] = z;
  }
  // L^T lambda = z: lambda_j = z_j - l_{j+1} lambda_{j+1}, l_{j+1} = hm rd_j on rows < n
  auto lnext = [&](int j) {
    const bool ok = wok && k0 + 2 * (j + 1) < n;
    return ok ? hm * rdj[j] : 0.0;
  };
  double T = 1.0;
  double2 lp = zero2();
#pragma unroll
  for (int j = C - 1; j >= 0; --j) {
    const double l = lnext(j);
    const double2 v = c_fnms(l, lp, x[j]);
    x[j] = v;
    lp = v;
    T *= -l;
  }
  double sT = T;
  double2 sb = lp;
  auto lvlb = [&](auto dd) {
    constexpr int D = decltype(dd)::value;
    const double oT = chain_hi<G, D>(sT, m);
    const double2 ob = chain_hi<G, D>(sb, m);
    sb = c_fma(sT, ob, sb);
    sT = sT * oT;
  };
  lvlb(std::integral_constant<int, 1>{});
  if constexpr (G > 2) lvlb(std::integral_constant<int, 2>{});
  if constexpr (G > 4) lvlb(std::integral_constant<int, 4>{});
  if constexpr (G > 8) lvlb(std::integral_constant<int, 8>{});
  if constexpr (G > 16) lvlb(std::integral_constant<int, 16>{});
  double2 h = chain_hi<G, 1>(sb, m);
#pragma unroll
  for (int j = C - 1; j >= 0; --j) {
    h = c_mul(-lnext(j), h);
    x[j] = c_add(x[j], h);
  }
  if (grad != nullptr) {
    // -Re(lambda^H B u), (B u)_k = bd0 u_k - pi/2 (u_{k-2} + u_{k+2})
    const double2* urow = ufwd + (wok ? w : 0) * (int64_t)N;
    double2 uu[C];
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int k = k0 + 2 * j;
      uu[j] = (wok && k < n) ? urow[k] : zero2();
    }
    const double2 up = chain_lo<G, 1>(uu[C - 1], m), un = chain_hi<G, 1>(uu[0], m);
    double gs = 0.0;
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int k = k0 + 2 * j;
      const double2 um = (j == 0) ? up : uu[j == 0 ? 0 : j - 1];
      const double2 upn = (j == C - 1) ? un : uu[j == C - 1 ? 0 : j + 1];
      double2 bu = c_mul(helm_mass_diag(k, N, gl), uu[j]);
      bu = c_fnms(0.5 * kPi, c_add(um, upn), bu);
      const bool ok = wok && k < n;
      if (ok) gs -= x[j].x * bu.x + x[j].y * bu.y;
    }
#pragma unroll
    for (int d = 1; d < 2 * G; d <<= 1) gs += __shfl_xor(gs, d, 2 * G);
    if (wok && (lane % (2 * G)) == 0) grad[w] = gs;
  }
  if (wok) {
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int k = k0 + 2 * j;
      if (k < N) lrow[k] = (k < n) ? x[j] : zero2();
    }
  }
  if (info != nullptr) {
    int b = bad;
#pragma unroll
    for (int d = 1; d < 2 * G; d <<= 1) b = min(b, __shfl_xor(b, d, 2 * G));
    if (wok && (lane % (2 * G)) == 0) info[w] = (b == INT_MAX) ? 0 : b + 1;
  }
}

// =========================================================================
// Helmholtz, FP32 factor/solve + FP64 iterative refinement (wave layout)
// =========================================================================
// The FP32 factors (1/d, g) stay in registers; every refinement step solves
// the current FP64 residual in FP32 with the same scans as the FP64 solve,
// adds the correction to u in FP64 and forms the next residual f - H u in
// FP64 in the wave layout (neighbours by row shifts, the same-parity suffix
// sum by a suffix scan of chunk totals).  f is read once and u written once.

// Solves (in place) L U x = x in FP32 with stored factors: rd[j], gg[j] of
// chunk element j (0 on padding rows), rd_in = 1/d of the row before the chunk.
template <int C, int G>
__device__ __forceinline__ void helm_solve32(int lane, bool wok, int n, float hm, float rd_in, const float (&rd)[C],
                                             const float (&gg)[C], float2 (&x)[C]) {
  const int p = (lane / G) & 1, m = lane % G;
  const int k0 = 2 * m * C + p;
  auto lof = [&](int j) {
    const bool ok = wok && k0 + 2 * j < n;
    return ok ? hm * (j == 0 ? rd_in : rd[j == 0 ? 0 : j - 1]) : 0.0f;
  };
  float T = 1.0f;
  float2 yp = make_float2(0.0f, 0.0f);
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const float l = lof(j);
    const float2 y = cf_fma(-l, yp, x[j]);
    x[j] = y;
    yp = y;
    T *= -l;
  }
  float sT = T;
  float2 sb = yp, h;
  if constexpr (G == 16) {
    auto lvl = [&](auto sh) {
      using S = decltype(sh);
      const float oT = S::from_lower(sT);
      const float2 ob = S::from_lower(sb);
      sb = cf_fma(sT, ob, sb);
      sT = sT * oT;
    };
    lvl(RowShift<1>{});
    lvl(RowShift<2>{});
    lvl(RowShift<4>{});
    lvl(RowShift<8>{});
    h = RowShift<1>::from_lower(sb);
  } else {
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
      const float oT = __shfl_up(sT, (unsigned)d, G);
      const float2 ob = make_float2(__shfl_up(sb.x, (unsigned)d, G), __shfl_up(sb.y, (unsigned)d, G));
      if (m >= d) {
        sb = cf_fma(sT, ob, sb);
        sT = sT * oT;
      }
    }
    h = make_float2(__shfl_up(sb.x, 1u, G), __shfl_up(sb.y, 1u, G));
    if (m == 0) h = make_float2(0.0f, 0.0f);
  }
#pragma unroll
  for (int j = 0; j < C; ++j) {
    h = cf_mul(-lof(j), h);
    x[j] = cf_add(x[j], h);
  }
  float A00 = 1.0f, A01 = 0.0f, A10 = 0.0f, A11 = 1.0f;
  float2 c0 = make_float2(0.0f, 0.0f), c1 = make_float2(0.0f, 0.0f);
#pragma unroll
  for (int j = C - 1; j >= 0; --j) {
    const float r = rd[j];
    x[j] = cf_mul(r, x[j]);
    const float eh = r * (gg[j] + hm), gh = r * gg[j];
    const float n00 = -eh * A00 - gh * A10, n01 = -eh * A01 - gh * A11;
    const float n10 = A00 + A10, n11 = A01 + A11;
    A00 = n00;
    A01 = n01;
    A10 = n10;
    A11 = n11;
    float2 nc0 = cf_fma(-eh, c0, x[j]);
    nc0 = cf_fma(-gh, c1, nc0);
    const float2 nc1 = cf_add(c0, c1);
    c0 = nc0;
    c1 = nc1;
  }
  auto compose2 = [&](float o00, float o01, float o10, float o11, float2 oc0, float2 oc1) {
    const float2 n0 = cf_add(cf_fma(A00, oc0, cf_mul(A01, oc1)), c0);
    const float2 n1 = cf_add(cf_fma(A10, oc0, cf_mul(A11, oc1)), c1);
    const float n00 = A00 * o00 + A01 * o10, n01 = A00 * o01 + A01 * o11;
    const float n10 = A10 * o00 + A11 * o10, n11 = A10 * o01 + A11 * o11;
    A00 = n00;
    A01 = n01;
    A10 = n10;
    A11 = n11;
    c0 = n0;
    c1 = n1;
  };
  float2 sa, sS;
  if constexpr (G == 16) {
    auto lvl = [&](auto sh) {
      using S = decltype(sh);
      compose2(S::from_upper(A00), S::from_upper(A01), S::from_upper(A10), S::from_upper(A11), S::from_upper(c0),
               S::from_upper(c1));
    };
    lvl(RowShift<1>{});
    lvl(RowShift<2>{});
    lvl(RowShift<4>{});
    lvl(RowShift<8>{});
    sa = RowShift<1>::from_upper(c0);
    sS = RowShift<1>::from_upper(c1);
  } else {
    auto dn = [&](float v, int d) { return __shfl_down(v, (unsigned)d, G); };
    auto dn2 = [&](float2 v, int d) { return make_float2(dn(v.x, d), dn(v.y, d)); };
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
      const float o00 = dn(A00, d), o01 = dn(A01, d), o10 = dn(A10, d), o11 = dn(A11, d);
      const float2 oc0 = dn2(c0, d), oc1 = dn2(c1, d);
      if (m + d < G) compose2(o00, o01, o10, o11, oc0, oc1);
    }
    sa = dn2(c0, 1);
    sS = dn2(c1, 1);
    if (m == G - 1) {
      sa = make_float2(0.0f, 0.0f);
      sS = make_float2(0.0f, 0.0f);
    }
  }
#pragma unroll
  for (int j = C - 1; j >= 0; --j) {
    const float r = rd[j];
    const float eh = r * (gg[j] + hm), gh = r * gg[j];
    float2 uj = cf_fma(-eh, sa, x[j]);
    uj = cf_fma(-gh, sS, uj);
    x[j] = uj;
    sS = cf_add(sS, sa);
    sa = uj;
  }
}

// (H u)_k of this lane's chunk elements in FP64, handed to sink(j, hu) from
// the last element down: the banded part from the lane's own values and its
// neighbours' (row shifts), the same-parity tail from suffix sums of chunk
// totals.  u must be zero on padding rows.
template <int C, int G, typename Sink>
__device__ __forceinline__ void helm_apply(int N, int lane, double al, int gl, const double2 (&u)[C], Sink sink) {
  const int p = (lane / G) & 1, m = lane % G;
  const int k0 = 2 * m * C + p;
  double2 tot = zero2();
#pragma unroll
  for (int j = 0; j < C; ++j) tot = c_add(tot, u[j]);
  double2 u_prev, u_next, E;
  if constexpr (G == 16) {
    u_prev = RowShift<1>::from_lower(u[C - 1]);
    u_next = RowShift<1>::from_upper(u[0]);
    double2 inc = tot;  // inclusive suffix sum of chunk totals over lanes >= m
    inc = c_add(inc, RowShift<1>::from_upper(inc));
    inc = c_add(inc, RowShift<2>::from_upper(inc));
    inc = c_add(inc, RowShift<4>::from_upper(inc));
    inc = c_add(inc, RowShift<8>::from_upper(inc));
    E = RowShift<1>::from_upper(inc);
  } else {
    u_prev = shfl_up2(u[C - 1], 1, G);
    if (m == 0) u_prev = zero2();
    u_next = shfl_down2(u[0], 1, G);
    if (m == G - 1) u_next = zero2();
    double2 inc = tot;
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
      const double2 o = shfl_down2(inc, d, G);
      if (m + d < G) inc = c_add(inc, o);
    }
    E = shfl_down2(inc, 1, G);
    if (m == G - 1) E = zero2();
  }
  // R = suffix sum from element j+2 (rows >= k+4 of the chain, all lanes)
  double2 R2 = c_sub(E, u_next);  // from element C+1
  double2 R1 = E;                 // from element C
  const double hm = -0.5 * kPi * al;
#pragma unroll
  for (int j = C - 1; j >= 0; --j) {
    const int k = k0 + 2 * j;
    const HelmRow h = helm_row(k, al, N, gl);
    const double2 um = (j == 0) ? u_prev : u[j == 0 ? 0 : j - 1];
    const double2 up = (j == C - 1) ? u_next : u[j == C - 1 ? 0 : j + 1];
    double2 hu = c_mul(h.h0, u[j]);
    hu = c_fma(hm, um, hu);
    hu = c_fma(h.hpp + hm, up, hu);
    hu = c_fma(h.hpp, R2, hu);
    sink(j, hu);
    R2 = R1;
    R1 = c_add(R1, u[j]);
  }
}

// x = f - H u in FP64 (rounded to FP32 on output), 0 on padding rows.
template <int C, int G>
__device__ __forceinline__ void helm_residual(int N, int lane, bool wok, double al, int gl, const double2 (&f)[C],
                                              const double2 (&u)[C], float2 (&x)[C]) {
  const int n = N - 2;
  const int k0 = 2 * (lane % G) * C + ((lane / G) & 1);
  helm_apply<C, G>(N, lane, al, gl, u, [&](int j, double2 hu) {
    const bool ok = wok && k0 + 2 * j < n;
    x[j] = ok ? to_f2(c_sub(f[j], hu)) : make_float2(0.0f, 0.0f);
  });
}

// Reduction over the 2G lanes of a system.
template <int G>
__device__ __forceinline__ double sys_max(double v) {
#pragma unroll
  for (int d = 1; d < 2 * G; d <<= 1) v = fmax(v, __shfl_xor(v, d, 2 * G));
  return v;
}

template <int C, int G>
__global__ __launch_bounds__(64) void helm_mixed_wave(int N, int64_t nsys, const double* __restrict__ alpha,
                                                      const double2* __restrict__ f, double2* __restrict__ u, int gl,
                                                      int32_t* __restrict__ info, int32_t* __restrict__ iters, int it_max,
                                                      double tol) {
  constexpr int SPW = 64 / (2 * G);
  __shared__ double2 st64[64];
  const int lane = threadIdx.x & 63;
  const int sl = lane / (2 * G), p = (lane / G) & 1, m = lane % G;
  const int64_t w = (int64_t)blockIdx.x * SPW + sl;
  const bool wok = w < nsys;
  const int n = N - 2;
  const int k0 = 2 * m * C + p;
  const double al = wok ? alpha[w] : 0.0;
  const double2* frow = f + (wok ? w : 0) * (int64_t)N;
  double2* urow = u + (wok ? w : 0) * (int64_t)N;
  HelmPrev32 pv = {0.0f, 0.0f};
  if (wok && m > 0 && k0 < n) {
    const float2 s2 = reinterpret_cast<const float2*>(urow)[p * G + m];
    pv.rd = s2.x;
    pv.g = s2.y;
  }
  double2 fx[C];
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int k = k0 + 2 * j;
    fx[j] = (wok && k < n) ? frow[k] : zero2();
  }
  // FP32 factorisation
  const float hm32 = (float)(-0.5 * kPi * al);
  const float rd_in = (k0 >= 2) ? pv.rd : 0.0f;
  float rd[C], gg[C];
  bool finite32 = true;
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int k = k0 + 2 * j;
    const bool ok = wok && k < n;
    float l, g, r, d;
    helm_step32(k, al, N, gl, pv, l, g, r, d);
    pv.rd = r;
    pv.g = g;
    rd[j] = ok ? r : 0.0f;
    gg[j] = ok ? g : 0.0f;
    if (ok && !(fabsf(d) > 0.0f && fabsf(d) < 3.0e38f && fabsf(r) < 3.0e38f)) finite32 = false;
  }
  // refinement
  double2 ux[C];
  float2 x[C];
#pragma unroll
  for (int j = 0; j < C; ++j) {
    ux[j] = zero2();
    x[j] = to_f2(fx[j]);
  }
  bool running = wok && (sys_max<G>(finite32 ? 0.0 : 1.0) == 0.0);
  bool conv = false;
  double prev = 1e300;
  int ncorr = 0;
  for (int it = 0; it <= it_max; ++it) {  // the first solve, then it_max corrections at most
    helm_solve32<C, G>(lane, wok, n, hm32, rd_in, rd, gg, x);
    double dmax = 0.0, umax = 0.0;
#pragma unroll
    for (int j = 0; j < C; ++j) {
      if (running) ux[j] = c_add(ux[j], to_d2(x[j]));
      dmax = fmax(dmax, cabs1(to_d2(x[j])));
      umax = fmax(umax, cabs1(ux[j]));
    }
    dmax = sys_max<G>(dmax);
    umax = sys_max<G>(umax);
    if (running) {
      ncorr = it;
      refine_decide(it, it_max, dmax, umax, prev, tol, running, conv);
    }
    if (!__any(running)) break;
    helm_residual<C, G>(N, lane, wok, al, gl, fx, ux, x);
  }
  const bool failed = wok && !conv;
  int bad = INT_MAX;
  if (__any(failed)) {
    // FP64 re-solve of this wavefront's systems: restart states by one
    // sequential walk per chain (lane m = 0), then the FP64 wave solve
    if (m == 0 && wok) {
      const int nc = (n - p + 1) / 2;
      const int nchunks = (nc + C - 1) / C;
      HelmPrev q = {0.0, 0.0};
      for (int i = 0; i < (nchunks - 1) * C; ++i) {
        double l, g, r, d;
        helm_step(2 * i + p, al, N, gl, q, l, g, r, d);
        q.rd = r;
        q.g = g;
        if ((i + 1) % C == 0) st64[sl * 2 * G + p * G + (i + 1) / C] = make_double2(q.rd, q.g);
      }
    }
    __syncthreads();
    HelmPrev q = {0.0, 0.0};
    if (wok && m > 0 && k0 < n) {
      q.rd = st64[lane].x;
      q.g = st64[lane].y;
    }
    double2 x64[C];
#pragma unroll
    for (int j = 0; j < C; ++j) x64[j] = fx[j];
    bad = helm_wave_core<C, G, true>(N, lane, w, wok, al, q, x64, urow, gl, nullptr);
    if (failed) {
#pragma unroll
      for (int j = 0; j < C; ++j) ux[j] = x64[j];
    }
  }
  if (wok) {
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int k = k0 + 2 * j;
      if (k < N) urow[k] = (k < n) ? ux[j] : zero2();
    }
  }
  if (info != nullptr) {
    int b = failed ? bad : INT_MAX;
#pragma unroll
    for (int d = 1; d < 2 * G; d <<= 1) b = min(b, __shfl_xor(b, d, 2 * G));
    if (wok && (lane % (2 * G)) == 0) info[w] = failed ? (b == INT_MAX ? SHEN_INFO_REFINE_FALLBACK : b + 1) : 0;
  }
  if (iters != nullptr && wok && (lane % (2 * G)) == 0) iters[w] = ncorr;
}

// =========================================================================
// Biharmonic wave solve
// =========================================================================
struct NoHook {
  __device__ void operator()() const {}
};
// A fetch functor with a true static member `lazy` also serves the first
// forward sweep: f is then read as the sweep goes, not held from the start.
template <typename F, typename = void>
struct LazyFetch : std::false_type {};
template <typename F>
struct LazyFetch<F, std::void_t<decltype(F::lazy)>> : std::bool_constant<F::lazy> {};
template <int C, int G, bool PIPE = false, bool TAB = false, typename FetchF, typename Hook = NoHook, bool WALKINFO = false,
          typename Carry = NoCarry, int TP = 0>
__device__ __forceinline__ int bih_wave_core(int N, int lane, int64_t w, bool wok, double a, double b, BihRowState m2,
                                              BihRowState m4, double2 (&x)[C], FetchF fetch_f, double2* __restrict__ urow,
                                              int gl, int32_t* __restrict__ info, const double* tab, Hook after_f = Hook(),
                                              std::bool_constant<WALKINFO> = {}, int walk_bad = INT_MAX, Carry cy = Carry());

template <int C, int G, bool TAB = false>
__device__ __forceinline__ void bih_wave_body(int N, int64_t nsys, int64_t wbase, const double* __restrict__ ca,
                                              const double* __restrict__ cb, const double2* __restrict__ f,
                                              double2* __restrict__ u, const double2* __restrict__ sts, int64_t sstride,
                                              int gl, int32_t* __restrict__ info, const double* tab = nullptr) {
  int lane = threadIdx.x & 63;  // opaque, as in helm_wave_body
  asm volatile("" : "+v"(lane));
  lane &= 63;  // opaque, but known to be a lane index
  const int sl = lane / (2 * G);
  const int p = (lane / G) & 1;
  const int m = lane % G;
  const int64_t w = wbase + sl;
  const bool wok = w < nsys;
  const int n = N - 4;
  const int k0 = 2 * m * C + p;
  const double a = wok ? ca[w] : 0.0, b = wok ? cb[w] : 0.0;
  const double2* frow = f + (wok ? w : 0) * (int64_t)N;
  double2* urow = u + (wok ? w : 0) * (int64_t)N;

  BihRowState m2 = {0, 0, 0, 0, 0}, m4 = {0, 0, 0, 0, 0};
  if (wok && m > 0 && k0 < n) {
    const double2* s = sts + w * sstride + (p * G + m) * 5;
    const double2 s0 = s[0], s1 = s[1], s2 = s[2], s3 = s[3], s4 = s[4];
    m2 = BihRowState{s0.x, s0.y, s1.x, s1.y, s2.x};
    m4 = BihRowState{s2.y, s3.x, s3.y, s4.x, s4.y};
  }
  // the table-driven walk has checked the pivots (slot of chunk 0)
  int wb = INT_MAX;
  if (TAB && wok && m == 0) wb = walk_bad_of(sts[w * sstride + p * G * 5].x, true);
  double2 x[C];
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int k = k0 + 2 * j;
    x[j] = (wok && k < n) ? frow[k] : zero2();
  }
  auto fetch = [&](int j) {
    const int k = k0 + 2 * j;
    return (wok && k < n) ? frow[k] : zero2();
  };
  bih_wave_core<C, G, false, TAB>(N, lane, w, wok, a, b, m2, m4, x, fetch, urow, gl, info, tab, NoHook(),
                                  std::bool_constant<TAB>{}, wb);
}

// Everything after the loads: x holds f of this lane's chunk (0 where k >= n),
// m2/m4 the restart state, fetch_f(j) gives f of chunk element j again (the
// forward refinement sweep).  Without PIPE the solution is stored to urow;
// with PIPE it is left in x for the caller.
// WALKINFO: the boundary walk has already checked every pivot of the chain
// (it runs the same factorisation) and walk_bad holds, on the lanes of chunk
// 0, the first unusable row of the lane's chain (INT_MAX: none); the rows of
// the chunk are then not checked again.
template <int C, int G, bool PIPE, bool TAB, typename FetchF, typename Hook, bool WALKINFO, typename Carry, int TP>
__device__ __forceinline__ int bih_wave_core(int N, int lane, int64_t w, bool wok, double a, double b, BihRowState m2,
                                              BihRowState m4, double2 (&x)[C], FetchF fetch_f, double2* __restrict__ urow,
                                              int gl, int32_t* __restrict__ info, const double* tab, Hook after_f,
                                              std::bool_constant<WALKINFO>, int walk_bad, Carry cy) {
  const int hf = (lane / G) & 1;  // which G-lane half of the 2G lanes
  const int p = cy.parity(hf);    // the parity of this lane's chain
  const int m = lane % G;
  const int n = N - 4;
  const int k0 = cy.kbase(C, G, hf) + 2 * m * C + p;
  // factorisation restart + local forward elimination; keep normalised U rows
  constexpr int RT = 2 * G * C;
  double l1j[C], l2j[C], r0j[C], u2j[C], u4j[C], pj[C], rj[C];
  double q4j[TAB ? 1 : C];
  // q_{k+4}, s_{k+4} of chunk element j (backward passes)
  auto qs_of = [&](int j) {
    if constexpr (TAB) return bih_tab_qs(tab, C, k0 + 2 * j);
    const double k6 = (double)(k0 + 2 * j) + 6.0;
    return make_double2(q4j[TAB ? 0 : j], k6 * k6 * q4j[TAB ? 0 : j]);
  };
  int bad = WALKINFO ? walk_bad : INT_MAX;
  double T00 = 1.0, T01 = 0.0, T10 = 0.0, T11 = 1.0;
  double2 y1 = zero2(), y2 = zero2();  // y_{i-1}, y_{i-2}
  Recip Rc;
  BihConst cm2, cm4;
  if constexpr (TAB) {
    cm2 = bih_const_at<TP>(tab, RT, C, k0 - 2, N, gl);
    cm4 = bih_const_at<TP>(tab, RT, C, k0 - 4, N, gl);
  } else {
    Rc.init(k0);
  }
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int k = k0 + 2 * j;
    const bool ok = wok && k < n;
    BihRowState o;
    double l1, l2, t0, sc;
    if constexpr (TAB) {
      const BihConst c = bih_tab_get<TP>(tab, RT, C, k);
      bih_step_row(bih_row_tab(k, a, b, c, cm2.B2, cm2.q4, cm2.s4, cm4.B4), m2, m4, o, l1, l2, t0, sc);
      cm4 = cm2;
      cm2 = c;
    } else {
      if (j > 0) Rc.advance(k);
      bih_step(k, a, b, N, gl, Rc, m2, m4, o, l1, l2, t0, sc);
      q4j[TAB ? 0 : j] = Rc.p7;  // q_{k+4} = 1/(k+7)
    }
    if constexpr (!WALKINFO) {
      bad = first_bad(bad, ok && bad_pivot(t0, sc), k);
    }
    m4 = m2;
    m2 = o;
    // Table rows past the system are identity rows (zero l, unit pivot, no
    // coupling), so only the computed-row path masks them.
    auto keep = [&](double v) {
      if constexpr (TAB) return v;
      return ok ? v : 0.0;
    };
    l1 = keep(l1);
    l2 = keep(l2);
    l1j[j] = l1;
    l2j[j] = l2;
    r0j[j] = keep(o.rU0);
    u2j[j] = keep(o.rU0 * o.U2);
    u4j[j] = keep(o.rU0 * o.U4);
    pj[j] = keep(o.rU0 * o.P);
    rj[j] = keep(o.rU0 * o.R);
    double2 fj;
    if constexpr (LazyFetch<FetchF>::value) {
      fj = fetch_f(j);
    } else {
      fj = x[j];
    }
    double2 y = c_fnms(l1, y1, fj);
    y = c_fnms(l2, y2, y);
    x[j] = y;
    y2 = y1;
    y1 = y;
    // T <- [[-l1, -l2],[1, 0]] T
    const double n00 = -l1 * T00 - l2 * T10, n01 = -l1 * T01 - l2 * T11;
    T10 = T00;
    T11 = T01;
    T00 = n00;
    T01 = n01;
  }
  // settle the pivot checks here: sunk to their only use at the end, they
  // would keep every row's pivot and scale live through both sweeps
  if constexpr (!WALKINFO) asm volatile("" : "+v"(bad));
  // forward scan: (T, b = (y_last, y_last-1)); compose(later, earlier) = (T_l T_e, T_l b_e + b_l)
  const double L00 = T00, L01 = T01, L10 = T10, L11 = T11;  // this chunk's own transfer
  double2 b0 = y1, b1 = y2;
  auto composeT = [&](double o00, double o01, double o10, double o11, double2 ob0, double2 ob1) {
    const double2 n0 = c_add(c_fma(T00, ob0, c_mul(T01, ob1)), b0);
    const double2 n1 = c_add(c_fma(T10, ob0, c_mul(T11, ob1)), b1);
    const double n00 = T00 * o00 + T01 * o10, n01 = T00 * o01 + T01 * o11;
    const double n10 = T10 * o00 + T11 * o10, n11 = T10 * o01 + T11 * o11;
    T00 = n00;
    T01 = n01;
    T10 = n10;
    T11 = n11;
    b0 = n0;
    b1 = n1;
  };
  double2 h1, h2;
  // Prefix scan of the chunk maps across the chain; afterwards (h1, h2) is
  // the state entering this chunk.  G = 16: one DPP row per chain.  G = 32:
  // the same within each row, then the upper row completes its prefixes with
  // the lower row's total (lane 15), which is also the state entering lane 16.
  auto fscan = [&]() {
    if constexpr ((G == 16 || G == 32) && !Carry::on) {
      auto lvl = [&](auto sh) {
        using S = decltype(sh);
        if constexpr (G == 32) {
          composeT(S::from_lower_one(T00), S::from_lower(T01), S::from_lower(T10), S::from_lower_one(T11),
                   S::from_lower(b0), S::from_lower(b1));
        } else {
          composeT(S::from_lower(T00), S::from_lower(T01), S::from_lower(T10), S::from_lower(T11), S::from_lower(b0),
                   S::from_lower(b1));
        }
      };
      lvl(RowShift<1>{});
      lvl(RowShift<2>{});
      lvl(RowShift<4>{});
      lvl(RowShift<8>{});
      if constexpr (G == 32) {
        // (T is now this lane's prefix within its row: missing partners
        // composed as the identity)
        const double2 t0 = chain_lane32<15>(b0, hf), t1 = chain_lane32<15>(b1, hf);
        const double2 n0 = c_add(c_fma(T00, t0, c_mul(T01, t1)), b0);
        const double2 n1 = c_add(c_fma(T10, t0, c_mul(T11, t1)), b1);
        b0 = c_sel(m >= 16, n0, b0);
        b1 = c_sel(m >= 16, n1, b1);
        const double2 s0 = RowShift<1>::from_lower(b0), s1 = RowShift<1>::from_lower(b1);
        h1 = c_sel(m == 16, t0, s0);
        h2 = c_sel(m == 16, t1, s1);
      } else {
        h1 = RowShift<1>::from_lower(b0);
        h2 = RowShift<1>::from_lower(b1);
      }
    } else {
#pragma unroll
      for (int d = 1; d < G; d <<= 1) {
        const double o00 = shfl_up_w(T00, d, G), o01 = shfl_up_w(T01, d, G);
        const double o10 = shfl_up_w(T10, d, G), o11 = shfl_up_w(T11, d, G);
        const double2 ob0 = shfl_up2(b0, d, G), ob1 = shfl_up2(b1, d, G);
        if (m >= d) composeT(o00, o01, o10, o11, ob0, ob1);
      }
      h1 = shfl_up2(b0, 1, G);
      h2 = shfl_up2(b1, 1, G);
      if (m == 0) {
        h1 = zero2();
        h2 = zero2();
      }
    }
  };
  fscan();
  // with chains across wavefronts: the state entering this wavefront's
  // segment, hence this lane's, and the state entering the next lane (cn)
  double2 cn1 = zero2(), cn2 = zero2();
  if constexpr (Carry::on) {
    const double M[2][2] = {{T00, T01}, {T10, T11}};
    const double2 c[2] = {b0, b1};
    double2 sin[2];
    cy.template fold<2, false>(0, hf, m == G - 1, M, c, sin);
    cn1 = c_add(c_fma(T00, sin[0], c_mul(T01, sin[1])), b0);
    cn2 = c_add(c_fma(T10, sin[0], c_mul(T11, sin[1])), b1);
    h1 = c_sel(m == 0, sin[0], shfl_up2(cn1, 1, G));
    h2 = c_sel(m == 0, sin[1], shfl_up2(cn2, 1, G));
  }
  // The chunk-local particular solutions started from a zero state can be far
  // larger than y itself (the forward recurrence has modes of modulus close to
  // one), so the scanned incoming states carry their rounding.  One refinement
  // sweep: rerun every chunk from f and the scanned state sh, scan the (small)
  // defects e_m - sh_{m+1} with the same transfers, and add the response.
  const double2 sh1 = h1, sh2 = h2;  // approximate (y_{i0-1}, y_{i0-2})
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const double2 fj = fetch_f(j);
    double2 y = c_fnms(l1j[j], h1, fj);
    y = c_fnms(l2j[j], h2, y);
    x[j] = y;
    h2 = h1;
    h1 = y;
  }
  after_f();  // f is not read again
  {
    double2 nx1, nx2;  // approximate incoming state of the next chunk
    if constexpr (Carry::on) {
      nx1 = cn1;
      nx2 = cn2;
    } else if constexpr (G == 16) {
      nx1 = RowShift<1>::from_upper(sh1);
      nx2 = RowShift<1>::from_upper(sh2);
    } else if constexpr (G == 32) {
      const double2 u1 = RowShift<1>::from_upper(sh1), u2 = RowShift<1>::from_upper(sh2);
      const double2 c1 = chain_lane32<16>(sh1, hf), c2 = chain_lane32<16>(sh2, hf);
      nx1 = c_sel(m == 15, c1, u1);
      nx2 = c_sel(m == 15, c2, u2);
    } else {
      nx1 = shfl_down2(sh1, 1, G);
      nx2 = shfl_down2(sh2, 1, G);
    }
    T00 = L00;
    T01 = L01;
    T10 = L10;
    T11 = L11;
    b0 = c_sub(h1, nx1);
    b1 = c_sub(h2, nx2);
  }
  fscan();
  if constexpr (Carry::on) {  // the correction entering this wavefront's segment, then this lane
    const double M[2][2] = {{T00, T01}, {T10, T11}};
    const double2 c[2] = {b0, b1};
    double2 din[2];
    cy.template fold<2, false>(1, hf, m == G - 1, M, c, din);
    const double2 e1 = c_add(c_fma(T00, din[0], c_mul(T01, din[1])), b0);
    const double2 e2 = c_add(c_fma(T10, din[0], c_mul(T11, din[1])), b1);
    h1 = c_sel(m == 0, din[0], shfl_up2(e1, 1, G));
    h2 = c_sel(m == 0, din[1], shfl_up2(e2, 1, G));
  }
#pragma unroll
  for (int j = 0; j < C; ++j) {
    double2 hj = c_mul(-l1j[j], h1);
    hj = c_fma(-l2j[j], h2, hj);
    x[j] = c_mul(r0j[j], c_add(x[j], hj));  // yh
    h2 = h1;
    h1 = hj;
  }
  // backward: state s = (a = u_{i+1}, bb = u_{i+2}, cq = sq_{i+3}, cs = ss_{i+3})
  //   u_i = yh - u2h a - u4h bb - ph cq - rh cs ;  s' = (u_i, a, cq + q4 bb, cs + s4 bb)
  double A[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) A[r][c] = (r == c) ? 1.0 : 0.0;
  double2 cv[4] = {zero2(), zero2(), zero2(), zero2()};
#pragma unroll
  for (int j = C - 1; j >= 0; --j) {
    const double2 qs = qs_of(j);
    const double q4 = qs.x, s4 = qs.y;  // q_{k+4}, s_{k+4}
    double nA0[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
      nA0[c] = -(u2j[j] * A[0][c] + u4j[j] * A[1][c] + pj[j] * A[2][c] + rj[j] * A[3][c]);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double a1 = A[1][c];
      A[2][c] = __builtin_fma(q4, a1, A[2][c]);
      A[3][c] = __builtin_fma(s4, a1, A[3][c]);
      A[1][c] = A[0][c];
      A[0][c] = nA0[c];
    }
    double2 nc0 = c_fma(-u2j[j], cv[0], x[j]);
    nc0 = c_fma(-u4j[j], cv[1], nc0);
    nc0 = c_fma(-pj[j], cv[2], nc0);
    nc0 = c_fma(-rj[j], cv[3], nc0);
    cv[2] = c_fma(q4, cv[1], cv[2]);
    cv[3] = c_fma(s4, cv[1], cv[3]);
    cv[1] = cv[0];
    cv[0] = nc0;
  }
  // suffix scan: compose(lower, higher) = (A_lo A_hi, A_lo c_hi + c_lo)
  auto compose4 = [&](const double (&oA)[4][4], const double2 (&oc)[4]) {
    double nA[4][4];
    double2 ncv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double2 acc = cv[r];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc = c_fma(A[r][c], oc[c], acc);
      ncv[r] = acc;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < 4; ++t) s = __builtin_fma(A[r][t], oA[t][c], s);
        nA[r][c] = s;
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      cv[r] = ncv[r];
#pragma unroll
      for (int c = 0; c < 4; ++c) A[r][c] = nA[r][c];
    }
  };
  double2 sa, sb, sq, ss;
  if constexpr ((G == 16 || G == 32) && !Carry::on) {
    auto lvl = [&](auto sh) {
      using S = decltype(sh);
      double oA[4][4];
      double2 oc[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if constexpr (G == 32) {
            oA[r][c] = (r == c) ? S::from_upper_one(A[r][c]) : S::from_upper(A[r][c]);
          } else {
            oA[r][c] = S::from_upper(A[r][c]);
          }
        }
        oc[r] = S::from_upper(cv[r]);
      }
      compose4(oA, oc);
    };
    lvl(RowShift<1>{});
    lvl(RowShift<2>{});
    lvl(RowShift<4>{});
    lvl(RowShift<8>{});
    if constexpr (G == 32) {
      // the lower row completes its suffixes with the upper row's total
      // (lane 16, whose own suffix reaches the top of the chain), which is
      // also the state entering lane 15
      double2 t[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) t[r] = chain_lane32<16>(cv[r], hf);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double2 acc = cv[r];
#pragma unroll
        for (int c = 0; c < 4; ++c) acc = c_fma(A[r][c], t[c], acc);
        cv[r] = c_sel(m < 16, acc, cv[r]);
      }
      const double2 s0 = RowShift<1>::from_upper(cv[0]), s1 = RowShift<1>::from_upper(cv[1]);
      const double2 s2 = RowShift<1>::from_upper(cv[2]), s3 = RowShift<1>::from_upper(cv[3]);
      sa = c_sel(m == 15, t[0], s0);
      sb = c_sel(m == 15, t[1], s1);
      sq = c_sel(m == 15, t[2], s2);
      ss = c_sel(m == 15, t[3], s3);
    } else {
      sa = RowShift<1>::from_upper(cv[0]);
      sb = RowShift<1>::from_upper(cv[1]);
      sq = RowShift<1>::from_upper(cv[2]);
      ss = RowShift<1>::from_upper(cv[3]);
    }
  } else {
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
      double oA[4][4];
      double2 oc[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
#pragma unroll
        for (int c = 0; c < 4; ++c) oA[r][c] = shfl_down_w(A[r][c], d, G);
        oc[r] = shfl_down2(cv[r], d, G);
      }
      if (m + d < G) compose4(oA, oc);
    }
    if constexpr (Carry::on) {  // the state entering this wavefront's segment from above, then this lane
      double2 top[4], y[4];
      cy.template fold<4, true>(2, hf, m == 0, A, cv, top);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double2 acc = cv[r];
#pragma unroll
        for (int c = 0; c < 4; ++c) acc = c_fma(A[r][c], top[c], acc);
        y[r] = acc;
      }
      sa = c_sel(m == G - 1, top[0], shfl_down2(y[0], 1, G));
      sb = c_sel(m == G - 1, top[1], shfl_down2(y[1], 1, G));
      sq = c_sel(m == G - 1, top[2], shfl_down2(y[2], 1, G));
      ss = c_sel(m == G - 1, top[3], shfl_down2(y[3], 1, G));
    } else {
      sa = shfl_down2(cv[0], 1, G);
      sb = shfl_down2(cv[1], 1, G);
      sq = shfl_down2(cv[2], 1, G);
      ss = shfl_down2(cv[3], 1, G);
      if (m == G - 1) {
        sa = zero2();
        sb = zero2();
        sq = zero2();
        ss = zero2();
      }
    }
  }
#pragma unroll
  for (int j = C - 1; j >= 0; --j) {
    double2 uj = c_fma(-u2j[j], sa, x[j]);
    uj = c_fma(-u4j[j], sb, uj);
    uj = c_fma(-pj[j], sq, uj);
    uj = c_fma(-rj[j], ss, uj);
    x[j] = uj;
    const double2 qs = qs_of(j);
    sq = c_fma(qs.x, sb, sq);
    ss = c_fma(qs.y, sb, ss);
    sb = sa;
    sa = uj;
  }
  if constexpr (!PIPE) {
    if (wok) {
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const int k = k0 + 2 * j;
        if (k < N) urow[k] = (TAB || k < n) ? x[j] : zero2();  // table rows past n solve to zero
      }
    }
  }
  if (info != nullptr) {
    int bq = bad;
#pragma unroll
    for (int d = 1; d < 2 * G; d <<= 1) bq = min(bq, __shfl_xor(bq, d, 2 * G));
    if (wok && (lane % (2 * G)) == 0) info[w] = (bq == INT_MAX) ? 0 : bq + 1;
  }
  return bad;
}

template <int C, int G>
__global__ __launch_bounds__(64) void helm_wave_solve(int N, int64_t nsys, const double* __restrict__ alpha,
                                                      const double2* __restrict__ f, double2* __restrict__ u,
                                                      const double2* __restrict__ sts, int64_t sstride, int gl,
                                                      int32_t* __restrict__ info) {
  constexpr int SPW = 64 / (2 * G);
  helm_wave_body<C, G>(N, nsys, (int64_t)blockIdx.x * SPW, alpha, f, u, sts, sstride, gl, info);
}

// =========================================================================
// Biharmonic, FP32 factor/solve + FP64 iterative refinement (wave layout)
// =========================================================================
// Factors of the FP32 solve, per chunk element (0 on padding rows).
template <int C>
struct BihFac32 {
  float l1[C], l2[C], r0[C], u2[C], u4[C], p[C], r[C];
};

// In place: x <- H^{-1} x in FP32 with stored factors (the FP64 wave solve's
// scans, without the forward refinement sweep).
template <int C, int G>
__device__ __forceinline__ void bih_solve32(int lane, const BihFac32<C>& F, const double* tab, float2 (&x)[C]) {
  const int p = (lane / G) & 1, m = lane % G;
  const int k0 = 2 * m * C + p;
  float T00 = 1.0f, T01 = 0.0f, T10 = 0.0f, T11 = 1.0f;
  float2 y1 = make_float2(0.0f, 0.0f), y2 = y1;
#pragma unroll
  for (int j = 0; j < C; ++j) {
    float2 y = cf_fma(-F.l1[j], y1, x[j]);
    y = cf_fma(-F.l2[j], y2, y);
    x[j] = y;
    y2 = y1;
    y1 = y;
    const float n00 = -F.l1[j] * T00 - F.l2[j] * T10, n01 = -F.l1[j] * T01 - F.l2[j] * T11;
    T10 = T00;
    T11 = T01;
    T00 = n00;
    T01 = n01;
  }
  float2 b0 = y1, b1 = y2;
  auto composeT = [&](float o00, float o01, float o10, float o11, float2 ob0, float2 ob1) {
    const float2 n0 = cf_add(cf_fma(T00, ob0, cf_mul(T01, ob1)), b0);
    const float2 n1 = cf_add(cf_fma(T10, ob0, cf_mul(T11, ob1)), b1);
    const float n00 = T00 * o00 + T01 * o10, n01 = T00 * o01 + T01 * o11;
    const float n10 = T10 * o00 + T11 * o10, n11 = T10 * o01 + T11 * o11;
    T00 = n00;
    T01 = n01;
    T10 = n10;
    T11 = n11;
    b0 = n0;
    b1 = n1;
  };
  auto lvlT = [&](auto dd) {
    constexpr int D = decltype(dd)::value;
    const float o00 = chain_lo<G, D>(T00, m), o01 = chain_lo<G, D>(T01, m), o10 = chain_lo<G, D>(T10, m),
                o11 = chain_lo<G, D>(T11, m);
    const float2 ob0 = chain_lo<G, D>(b0, m), ob1 = chain_lo<G, D>(b1, m);
    composeT(o00, o01, o10, o11, ob0, ob1);
  };
  lvlT(std::integral_constant<int, 1>{});
  if constexpr (G > 2) lvlT(std::integral_constant<int, 2>{});
  if constexpr (G > 4) lvlT(std::integral_constant<int, 4>{});
  if constexpr (G > 8) lvlT(std::integral_constant<int, 8>{});
  if constexpr (G > 16) lvlT(std::integral_constant<int, 16>{});
  float2 h1 = chain_lo<G, 1>(b0, m), h2 = chain_lo<G, 1>(b1, m);
#pragma unroll
  for (int j = 0; j < C; ++j) {
    float2 hj = cf_mul(-F.l1[j], h1);
    hj = cf_fma(-F.l2[j], h2, hj);
    x[j] = cf_add(x[j], hj);
    h2 = h1;
    h1 = hj;
  }
  float A[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) A[r][c] = (r == c) ? 1.0f : 0.0f;
  float2 cv[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) cv[r] = make_float2(0.0f, 0.0f);
#pragma unroll
  for (int j = C - 1; j >= 0; --j) {
    const double2 qs = bih_tab_qs(tab, C, k0 + 2 * j);
    const float q4 = (float)qs.x, s4 = (float)qs.y;
    x[j] = cf_mul(F.r0[j], x[j]);
    float nA0[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) nA0[c] = -(F.u2[j] * A[0][c] + F.u4[j] * A[1][c] + F.p[j] * A[2][c] + F.r[j] * A[3][c]);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float a1 = A[1][c];
      A[2][c] = __builtin_fmaf(q4, a1, A[2][c]);
      A[3][c] = __builtin_fmaf(s4, a1, A[3][c]);
      A[1][c] = A[0][c];
      A[0][c] = nA0[c];
    }
    float2 nc0 = cf_fma(-F.u2[j], cv[0], x[j]);
    nc0 = cf_fma(-F.u4[j], cv[1], nc0);
    nc0 = cf_fma(-F.p[j], cv[2], nc0);
    nc0 = cf_fma(-F.r[j], cv[3], nc0);
    cv[2] = cf_fma(q4, cv[1], cv[2]);
    cv[3] = cf_fma(s4, cv[1], cv[3]);
    cv[1] = cv[0];
    cv[0] = nc0;
  }
  auto lvlA = [&](auto dd) {
    constexpr int D = decltype(dd)::value;
    float oA[4][4];
    float2 oc[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int c = 0; c < 4; ++c) oA[r][c] = chain_hi<G, D>(A[r][c], m);
      oc[r] = chain_hi<G, D>(cv[r], m);
    }
    float nA[4][4];
    float2 ncv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float2 acc = cv[r];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc = cf_fma(A[r][c], oc[c], acc);
      ncv[r] = acc;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        float t = 0.0f;
#pragma unroll
        for (int q = 0; q < 4; ++q) t = __builtin_fmaf(A[r][q], oA[q][c], t);
        nA[r][c] = t;
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      cv[r] = ncv[r];
#pragma unroll
      for (int c = 0; c < 4; ++c) A[r][c] = nA[r][c];
    }
  };
  lvlA(std::integral_constant<int, 1>{});
  if constexpr (G > 2) lvlA(std::integral_constant<int, 2>{});
  if constexpr (G > 4) lvlA(std::integral_constant<int, 4>{});
  if constexpr (G > 8) lvlA(std::integral_constant<int, 8>{});
  if constexpr (G > 16) lvlA(std::integral_constant<int, 16>{});
  float2 sa = chain_hi<G, 1>(cv[0], m), sb = chain_hi<G, 1>(cv[1], m), sq = chain_hi<G, 1>(cv[2], m),
         ss = chain_hi<G, 1>(cv[3], m);
#pragma unroll
  for (int j = C - 1; j >= 0; --j) {
    const double2 qs = bih_tab_qs(tab, C, k0 + 2 * j);
    float2 uj = cf_fma(-F.u2[j], sa, x[j]);
    uj = cf_fma(-F.u4[j], sb, uj);
    uj = cf_fma(-F.p[j], sq, uj);
    uj = cf_fma(-F.r[j], ss, uj);
    x[j] = uj;
    sq = cf_fma((float)qs.x, sb, sq);
    ss = cf_fma((float)qs.y, sb, ss);
    sb = sa;
    sa = uj;
  }
}

// (H u)_k of this lane's chunk elements in FP64, handed to sink(j, hu) from
// the last element down; rows from the table as in the factorisation.
// Walking the chunk downwards, each row's constants are read once and carried
// to the two rows below (which need them as those of rows k-2 and k-4);
// q_k, s_k are the table's q4, s4 of row k-4.  u must be zero on padding rows.
template <int C, int G, int TP = 0, typename Sink>
__device__ __forceinline__ void bih_apply(int N, int lane, double a, double b, int gl, const double* tab, const double2 (&u)[C],
                                          Sink sink) {
  constexpr int RT = 2 * G * C;
  const int p = (lane / G) & 1, m = lane % G;
  const int k0 = 2 * m * C + p;
  // constants of rows k0 + 2(C-1) and the two below it
  BihConst c = bih_const_at<TP>(tab, RT, C, k0 + 2 * (C - 1), N, gl);
  BihConst c2 = bih_const_at<TP>(tab, RT, C, k0 + 2 * (C - 2), N, gl);
  BihConst c4 = bih_const_at<TP>(tab, RT, C, k0 + 2 * (C - 3), N, gl);
  double2 TQ = zero2(), TS = zero2();
  {
    // q_k, s_k of every element: rows k-4 of the table
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const double2 qs = (j >= 2) ? bih_tab_qs(tab, C, k0 + 2 * (j - 2)) : make_double2(0.0, 0.0);
      const BihConst cn = bih_const_at<TP>(tab, RT, C, k0 + 2 * j - 4, N, gl);
      const double q = (j >= 2) ? qs.x : cn.q4, sv = (j >= 2) ? qs.y : cn.s4;
      TQ = c_fma(q, u[j], TQ);
      TS = c_fma(sv, u[j], TS);
    }
  }
  const double2 pl1 = chain_lo<G, 1>(u[C - 1], m), pl2 = chain_lo<G, 1>(u[C - 2], m);  // rows k0-2, k0-4
  const double2 nx1 = chain_hi<G, 1>(u[0], m), nx2 = chain_hi<G, 1>(u[1], m);          // rows k0+2C, k0+2C+2
  double2 iq = TQ, is = TS;  // inclusive suffix sums over lanes >= m
  auto lvl = [&](auto dd) {
    constexpr int D = decltype(dd)::value;
    iq = c_add(iq, chain_hi<G, D>(iq, m));
    is = c_add(is, chain_hi<G, D>(is, m));
  };
  lvl(std::integral_constant<int, 1>{});
  if constexpr (G > 2) lvl(std::integral_constant<int, 2>{});
  if constexpr (G > 4) lvl(std::integral_constant<int, 4>{});
  if constexpr (G > 8) lvl(std::integral_constant<int, 8>{});
  if constexpr (G > 16) lvl(std::integral_constant<int, 16>{});
  const double2 EQ = chain_hi<G, 1>(iq, m), ES = chain_hi<G, 1>(is, m);
  // q, s of rows k0+2C and k0+2C+2: q4, s4 of rows k0+2C-4 and k0+2C-2
  const double2 qs1 = bih_tab_qs(tab, C, k0 + 2 * C - 4), qs2 = bih_tab_qs(tab, C, k0 + 2 * C - 2);
  // sliding suffix sums from elements j+3, j+2, j+1 (rows >= k+6, k+4, k+2)
  double2 Q1 = EQ, S1 = ES;                                          // from element C
  double2 Q2 = c_fnms(qs1.x, nx1, EQ), S2 = c_fnms(qs1.y, nx1, ES);  // from element C+1
  double2 Q3 = c_fnms(qs2.x, nx2, Q2), S3 = c_fnms(qs2.y, nx2, S2);  // from element C+2
#pragma unroll
  for (int j = C - 1; j >= 0; --j) {
    const int k = k0 + 2 * j;
    // constants of row k-6 for the next step down (rows < 0: q4, s4 only)
    const BihConst c6 = bih_const_at<TP>(tab, RT, C, k - 6, N, gl);
    const BihRow h = bih_row_tab(k, a, b, c, c2.B2, c2.q4, c2.s4, c4.B4);
    const double2 um4 = (j >= 2) ? u[j >= 2 ? j - 2 : 0] : (j == 1 ? pl1 : pl2);
    const double2 um2 = (j >= 1) ? u[j >= 1 ? j - 1 : 0] : pl1;
    const double2 up2 = (j <= C - 2) ? u[j <= C - 2 ? j + 1 : 0] : nx1;
    const double2 up4 = (j <= C - 3) ? u[j <= C - 3 ? j + 2 : 0] : (j == C - 2 ? nx1 : nx2);
    double2 hu = c_mul(h.h0, u[j]);
    hu = c_fma(h.hm4, um4, hu);
    hu = c_fma(h.hm2, um2, hu);
    hu = c_fma(h.hp2, up2, hu);
    hu = c_fma(h.hp4, up4, hu);
    hu = c_fma(h.p, Q3, hu);
    hu = c_fma(h.r, S3, hu);
    sink(j, hu);
    const double q = c4.q4, sv = c4.s4;  // q_k, s_k
    Q3 = Q2;
    S3 = S2;
    Q2 = Q1;
    S2 = S1;
    Q1 = c_fma(q, u[j], Q1);
    S1 = c_fma(sv, u[j], S1);
    c = c2;
    c2 = c4;
    c4 = c6;
    // keep each row's table reads in its own step: hoisted ahead for all rows
    // they would hold some 11 registers per row
    asm volatile("" ::: "memory");
  }
}

// x = f - H u in FP64 (rounded to FP32 on output), 0 on padding rows.
template <int C, int G, int TP = 0, typename FetchF>
__device__ __forceinline__ void bih_residual(int N, int lane, bool wok, double a, double b, int gl, const double* tab,
                                             FetchF fetch_f, const double2 (&u)[C], float2 (&x)[C]) {
  const int n = N - 4;
  const int k0 = 2 * (lane % G) * C + ((lane / G) & 1);
  bih_apply<C, G, TP>(N, lane, a, b, gl, tab, u, [&](int j, double2 hu) {
    const bool ok = wok && k0 + 2 * j < n;
    x[j] = ok ? to_f2(c_sub(fetch_f(j), hu)) : make_float2(0.0f, 0.0f);
  });
}

// -------------------------------------------------------------------------
// Persistent, software-pipelined form of the wave solve (G >= 16, C >= 8).
//
// Each wavefront loops over groups of SPW = 64/(2G) systems.  Two LDS tiles
// per wavefront alternate: while one group is solved in registers, the next
// group's right-hand sides stream from HBM straight into the other tile
// (global_load_lds: no registers held, and each instruction covers 64
// consecutive rows, so HBM and L2 see whole lines); the solution leaves
// through the tile its group came in by, again as whole lines.
//
// Per iteration there is one wait on vector memory (after the arithmetic):
// then the prefetched tile is complete and the stores of the previous group
// are done, so the LDS traffic that follows (stage the solution, read the
// next group, read the staged rows back for the stores) runs with nothing
// outstanding, and only then is the tile refilled.
//
// Tile layout: system s, row k sits at entry 64 (s NB + k/64) + ((k mod 64)
// xor (m mod 16)), m = k / 2C its chunk, NB = 2GC/64.  Each global_load_lds
// instruction fills one 64-entry block; the xor spreads the 16 chunks that a
// group of 16 lanes touches at one step over all 16 bank groups.  NS extra
// 64-entry slots hold each lane's restart words.
// -------------------------------------------------------------------------
#define SHEN_LDS(ptr) ((__attribute__((address_space(3))) void*)(ptr))

template <int C, int G>
struct Tile {
  static constexpr int SPW = 64 / (2 * G);
  static constexpr int B = 2 * C;             // rows per chunk (both parities)
  static constexpr int NB = (2 * G * C) / 64;  // 64-row blocks per system
  static_assert(G >= 16 && C >= 8 && C % 4 == 0, "tile layout needs G >= 16 and C in {8, 16, ...}");
  // entry of row k of system s
  static __device__ __forceinline__ int pos(int s, int k) { return 64 * (s * NB + (k >> 6)) + ((k & 63) ^ ((k / B) & 15)); }
  // row held by entry (block i, lane l): the xor is an involution on the block
  static __device__ __forceinline__ int row(int i, int l) {
    const int t = i % NB;
    return 64 * t + (l ^ (((64 * t + l) / B) & 15));
  }
};

// Streams group g into tile T: C instructions of 64 consecutive rows each
// (rows >= N and systems >= nsys clamped to valid addresses; the reader masks
// them), then NS 16-byte restart words per lane from the state slots
// (system w's slot at sts + w sstride).
template <int C, int G, int NS>
__device__ __forceinline__ void prefetch_tile(double2* T, int lane, int64_t g, int N, int64_t nsys, const double2* __restrict__ f,
                                              const double2* __restrict__ sts, int64_t sstride) {
  using TL = Tile<C, G>;
#pragma unroll
  for (int i = 0; i < C; ++i) {
    const int s = i / TL::NB;
    const int64_t w = g * TL::SPW + s;
    const int64_t wc = w < nsys ? w : nsys - 1;
    const int k = TL::row(i, lane);
    const int kc = k < N ? k : N - 1;
    __builtin_amdgcn_global_load_lds((const void*)(f + wc * (int64_t)N + kc), SHEN_LDS(T + 64 * i), 16, 0, 0);
  }
  const int sl = lane / (2 * G), p = (lane / G) & 1, m = lane % G;
  const int64_t w = g * TL::SPW + sl;
  const int64_t wc = w < nsys ? w : nsys - 1;
  const double2* st = sts + wc * sstride + (p * G + m) * NS;
#pragma unroll
  for (int t = 0; t < NS; ++t)
    __builtin_amdgcn_global_load_lds((const void*)(st + t), SHEN_LDS(T + 64 * (C + t)), 16, 0, 0);
}

// f stays in LDS (one tile per wavefront, streamed in by LDS-DMA) where the
// layout allows it (G >= 16), else in registers.
template <int C, int G>
struct MixedTile {
  static constexpr size_t tile_bytes = (size_t)4 * C * 64 * sizeof(double2);
  static constexpr size_t base_bytes =
      (size_t)6 * 2 * G * C * sizeof(double2) + (size_t)4 * 64 * 10 * sizeof(double);
  // gfx950: 160 KiB of LDS per work group
  static constexpr bool value = (G >= 16 && C >= 8 && C % 4 == 0) && base_bytes + tile_bytes <= 160 * 1024;
  static constexpr size_t bytes = value ? tile_bytes : 0;
};

template <int C, int G>
__global__ __launch_bounds__(256) void bih_mixed_tab(int N, int64_t nsys, const double* __restrict__ ca,
                                                     const double* __restrict__ cb, const double2* __restrict__ f,
                                                     double2* __restrict__ u, int gl, int32_t* __restrict__ info,
                                                     int32_t* __restrict__ iters, int it_max, double tol) {
  constexpr int SPW = 64 / (2 * G);
  constexpr int RT = 2 * G * C;
  constexpr bool kTile = MixedTile<C, G>::value;
  extern __shared__ double smem[];
  const double* tab = smem;
  bih_tab_fill<6>(smem, RT, C, N, gl, threadIdx.x, 256);
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  double* st64 = smem + 2 * 6 * RT + wv * 64 * 10;  // FP64 restart states (fallback)
  double2* ftile = reinterpret_cast<double2*>(smem + 2 * 6 * RT + 4 * 64 * 10) + wv * (C * 64);
  const int lane = threadIdx.x & 63;
  const int sl = lane / (2 * G), p = (lane / G) & 1, m = lane % G;
  const int64_t g = (int64_t)blockIdx.x * 4 + wv;
  const int64_t w = g * SPW + sl;
  const bool wok = w < nsys;
  const int n = N - 4;
  const int k0 = 2 * m * C + p;
  if constexpr (kTile) prefetch_tile<C, G, 0>(ftile, lane, g, N, nsys, f, nullptr, 0);
  __syncthreads();  // the table
  const double a = wok ? ca[w] : 0.0, b = wok ? cb[w] : 0.0;
  const double2* frow = f + (wok ? w : 0) * (int64_t)N;
  double2* urow = u + (wok ? w : 0) * (int64_t)N;
  BihRowState32 m2 = {0, 0, 0, 0, 0}, m4 = {0, 0, 0, 0, 0};
  if (wok && m > 0 && k0 < n) {
    const float2* s = reinterpret_cast<const float2*>(urow) + (p * G + m) * 5;
    const float2 s0 = s[0], s1 = s[1], s2 = s[2], s3 = s[3], s4 = s[4];
    m2 = BihRowState32{s0.x, s0.y, s1.x, s1.y, s2.x};
    m4 = BihRowState32{s2.y, s3.x, s3.y, s4.x, s4.y};
  }
  // f of chunk element j (0 on padding rows)
  double2 fx[kTile ? 1 : C];
  if constexpr (kTile) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  } else {
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int k = k0 + 2 * j;
      fx[j] = (wok && k < n) ? frow[k] : zero2();
    }
  }
  auto fget = [&](int j) -> double2 {
    if constexpr (kTile) {
      using TL = Tile<C, G>;
      // tile positions from an opaque lane index at every use: kept from the
      // first use they were spilled
      int ln = threadIdx.x;
      asm volatile("" : "+v"(ln));
      ln &= 63;
      const int k = 2 * (ln % G) * C + ((ln / G) & 1) + 2 * j;
      const double2 v = ftile[TL::pos(ln / (2 * G), k)];
      return (wok && k < n) ? v : zero2();
    } else {
      return fx[kTile ? 0 : j];
    }
  };
  // FP32 factorisation
  BihFac32<C> F;
  bool finite32 = true;
  {
    BihConst cm2 = bih_const_at<6>(tab, RT, C, k0 - 2, N, gl), cm4 = bih_const_at<6>(tab, RT, C, k0 - 4, N, gl);
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int k = k0 + 2 * j;
      const bool ok = wok && k < n;
      const BihConst c = bih_tab_get<6>(tab, RT, C, k);
      BihRowState32 o;
      float l1, l2, t0;
      bih_step_row32(bih_row_tab(k, a, b, c, cm2.B2, cm2.q4, cm2.s4, cm4.B4), m2, m4, o, l1, l2, t0);
      cm4 = cm2;
      cm2 = c;
      m4 = m2;
      m2 = o;
      if (ok && !(fabsf(t0) > 0.0f && fabsf(t0) < 3.0e38f && fabsf(o.rU0) < 3.0e38f)) finite32 = false;
      F.l1[j] = ok ? l1 : 0.0f;
      F.l2[j] = ok ? l2 : 0.0f;
      F.r0[j] = ok ? o.rU0 : 0.0f;
      F.u2[j] = ok ? o.rU0 * o.U2 : 0.0f;
      F.u4[j] = ok ? o.rU0 * o.U4 : 0.0f;
      F.p[j] = ok ? o.rU0 * o.P : 0.0f;
      F.r[j] = ok ? o.rU0 * o.R : 0.0f;
    }
  }
  // refinement
  double2 ux[C];
  float2 x[C];
#pragma unroll
  for (int j = 0; j < C; ++j) {
    ux[j] = zero2();
    x[j] = to_f2(fget(j));
  }
  bool running = wok && (sys_max<G>(finite32 ? 0.0 : 1.0) == 0.0);
  bool conv = false;
  double prev = 1e300;
  int ncorr = 0;
  for (int it = 0; it <= it_max; ++it) {  // the first solve, then it_max corrections at most
    bih_solve32<C, G>(lane, F, tab, x);
    double dmax = 0.0, umax = 0.0;
#pragma unroll
    for (int j = 0; j < C; ++j) {
      if (running) ux[j] = c_add(ux[j], to_d2(x[j]));
      dmax = fmax(dmax, cabs1(to_d2(x[j])));
      umax = fmax(umax, cabs1(ux[j]));
    }
    dmax = sys_max<G>(dmax);
    umax = sys_max<G>(umax);
    if (running) {
      ncorr = it;
      refine_decide(it, it_max, dmax, umax, prev, tol, running, conv);
    }
    if (!__any(running)) break;
    bih_residual<C, G, 6>(N, lane, wok, a, b, gl, tab, fget, ux, x);
  }
  const bool failed = wok && !conv;
  // the refined solutions leave first, so that the FP64 re-solve below does
  // not hold them
  if (wok) {
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int k = k0 + 2 * j;
      if (k < N) urow[k] = (k < n) ? ux[j] : zero2();
    }
  }
  int bad = INT_MAX;
  if (__any(failed)) {
    // FP64 re-solve of this wavefront's systems: restart states by one
    // sequential walk per chain (lane m = 0) with the table rows, then the
    // FP64 wave solve with the same rows
    double* sts = st64 + sl * 2 * G * 10;
    if (m == 0 && wok) bih_walk_tab<C, G, false, 6>(N, p, a, b, sts, gl, tab);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    BihRowState q2 = {0, 0, 0, 0, 0}, q4 = {0, 0, 0, 0, 0};
    if (wok && m > 0 && k0 < n) {
      const double* sv = sts + (p * G + m) * 10;
      q2 = BihRowState{sv[0], sv[1], sv[2], sv[3], sv[4]};
      q4 = BihRowState{sv[5], sv[6], sv[7], sv[8], sv[9]};
    }
    double2 x64[C];
#pragma unroll
    for (int j = 0; j < C; ++j) x64[j] = fget(j);
    bad = bih_wave_core<C, G, true, true, decltype(fget), NoHook, false, NoCarry, 6>(N, lane, w, wok, a, b, q2, q4, x64, fget,
                                                                                     urow, gl, nullptr, tab);
    if (failed) {
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const int k = k0 + 2 * j;
        if (k < N) urow[k] = (k < n) ? x64[j] : zero2();
      }
    }
  }
  if (info != nullptr) {
    int bq = failed ? bad : INT_MAX;
#pragma unroll
    for (int d = 1; d < 2 * G; d <<= 1) bq = min(bq, __shfl_xor(bq, d, 2 * G));
    if (wok && (lane % (2 * G)) == 0) info[w] = failed ? (bq == INT_MAX ? SHEN_INFO_REFINE_FALLBACK : bq + 1) : 0;
  }
  if (iters != nullptr && wok && (lane % (2 * G)) == 0) iters[w] = ncorr;
}

// =========================================================================
// Biharmonic adjoint (wave layout): lambda = H^{-T} gbar and, when asked,
// grad_a = -Re(lambda^H A u), grad_b = -Re(lambda^H B u).  U^T z = gbar runs
// forward with the state (z_{j-1}, z_{j-2}, sum P_i z_i, sum R_i z_i over
// rows <= k-6), an affine 4x4 recurrence; L^T lambda = z runs backward with
// the state (lambda_{j+1}, lambda_{j+2}).  Rows from the LDS table, restart
// states from the table-driven boundary walk (parked in the lambda row).
// =========================================================================
// Whether bih_adjoint_tab keeps its reciprocal pivots in LDS as well as its
// multipliers (the row table of G = 32 leaves room for the multipliers only).
template <int G>
struct AdjR0Lds : std::bool_constant<(G <= 16)> {};

template <int C, int G>
__global__ __launch_bounds__(256) void bih_adjoint_tab(int N, int64_t nsys, const double* __restrict__ ca,
                                                       const double* __restrict__ cb, const double2* __restrict__ ufwd,
                                                       const double2* __restrict__ gbar, double2* __restrict__ lam,
                                                       const double2* __restrict__ sts, int64_t sstride,
                                                       double* __restrict__ grad_a, double* __restrict__ grad_b, int gl,
                                                       int32_t* __restrict__ info) {
  constexpr int SPW = 64 / (2 * G);
  constexpr int RT = 2 * G * C;
  extern __shared__ double tab[];
  bih_tab_fill(tab, RT, C, N, gl, threadIdx.x, 256);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int sl = lane / (2 * G), p = (lane / G) & 1, m = lane % G;
  const int64_t w = ((int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6))) * SPW + sl;
  const bool wok = w < nsys;
  const int n = N - 4;
  const int k0 = 2 * m * C + p;
  const double a = wok ? ca[w] : 0.0, b = wok ? cb[w] : 0.0;
  const double2* grow = gbar + (wok ? w : 0) * (int64_t)N;
  double2* lrow = lam + (wok ? w : 0) * (int64_t)N;
  BihRowState m2 = {0, 0, 0, 0, 0}, m4 = {0, 0, 0, 0, 0};
  if (wok && m > 0 && k0 < n) {
    const double2* sv = sts + w * sstride + (p * G + m) * 5;
    const double2 s0 = sv[0], s1 = sv[1], s2 = sv[2], s3 = sv[3], s4 = sv[4];
    m2 = BihRowState{s0.x, s0.y, s1.x, s1.y, s2.x};
    m4 = BihRowState{s2.y, s3.x, s3.y, s4.x, s4.y};
  }
  const BihRowState in2 = m2, in4 = m4;
  // gbar of chunk element j.  It is read twice (the local pass and the rerun)
  // rather than held in registers across the scan; the second read goes
  // through an opaque copy of the row pointer so that it is not merged with
  // the first.
  auto gload = [&](const double2* row, int j) {
    const int k = k0 + 2 * j;
    return (wok && k < n) ? row[k] : zero2();
  };
  double2 x[C];
  // factorisation restart (as the table-driven solve); raw U rows kept in
  // registers, the multipliers (used only by the L^T pass) in LDS after the
  // row table, element j of thread t at lmul[j * 256 + t]
  // Where the table leaves room (G <= 16), the reciprocal pivots follow them
  // (element j of thread t at r0l[j * 256 + t]).
  double2* lmul = reinterpret_cast<double2*>(tab + 2 * bih_tab_pairs(RT) * RT);
  constexpr bool kR0Lds = AdjR0Lds<G>::value;
  double* r0l = reinterpret_cast<double*>(lmul + C * 256);
  double r0j[kR0Lds ? 1 : C], u2j[C], u4j[C], pj[C], rj[C];
  auto R0 = [&](int j) {
    if constexpr (kR0Lds) return r0l[j * 256 + threadIdx.x];
    return r0j[kR0Lds ? 0 : j];
  };
  double l1_0 = 0.0, l2_0 = 0.0, l2_1 = 0.0;  // elements 0 and 1, for the neighbouring lane
  int bad = INT_MAX;
  {
    BihConst cm2 = bih_const_at(tab, RT, C, k0 - 2, N, gl), cm4 = bih_const_at(tab, RT, C, k0 - 4, N, gl);
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int k = k0 + 2 * j;
      const bool ok = wok && k < n;
      const BihConst c = bih_tab_get(tab, RT, C, k);
      BihRowState o;
      double l1, l2, t0, sc;
      bih_step_row(bih_row_tab(k, a, b, c, cm2.B2, cm2.q4, cm2.s4, cm4.B4), m2, m4, o, l1, l2, t0, sc);
      bad = first_bad(bad, ok && bad_pivot(t0, sc), k);
      cm4 = cm2;
      cm2 = c;
      m4 = m2;
      m2 = o;
      const double l1k = ok ? l1 : 0.0, l2k = ok ? l2 : 0.0;
      lmul[j * 256 + threadIdx.x] = make_double2(l1k, l2k);
      if (j == 0) {
        l1_0 = l1k;
        l2_0 = l2k;
      }
      if (j == 1) l2_1 = l2k;
      if constexpr (kR0Lds) {
        r0l[j * 256 + threadIdx.x] = ok ? o.rU0 : 0.0;
      } else {
        r0j[kR0Lds ? 0 : j] = ok ? o.rU0 : 0.0;
      }
      u2j[j] = ok ? o.U2 : 0.0;
      u4j[j] = ok ? o.U4 : 0.0;
      pj[j] = ok ? o.P : 0.0;
      rj[j] = ok ? o.R : 0.0;
    }
  }
  // the pivot checks are needed only at the end (info); settled here, or the
  // compiler keeps every row's pivot and scale live until then
  asm volatile("" : "+v"(bad));
  // coefficients of element j's forward step: U2 of row j-1, U4/P/R of row j-2
  auto U2p = [&](int j) { return j >= 1 ? u2j[j >= 1 ? j - 1 : 0] : in2.U2; };
  auto U4pp = [&](int j) { return j >= 2 ? u4j[j >= 2 ? j - 2 : 0] : (j == 1 ? in2.U4 : in4.U4); };
  auto Ppp = [&](int j) { return j >= 2 ? pj[j >= 2 ? j - 2 : 0] : (j == 1 ? in2.P : in4.P); };
  auto Rpp = [&](int j) { return j >= 2 ? rj[j >= 2 ? j - 2 : 0] : (j == 1 ? in2.R : in4.R); };
  auto qsj = [&](int j) {  // (q, s) of row k_j: q4, s4 of row k_j - 4
    const int k = k0 + 2 * j;
    if (j >= 2) return bih_tab_qs(tab, C, k - 4);  // k - 4 >= 0
    const BihConst c = bih_const_at(tab, RT, C, k - 4, N, gl);
    return make_double2(c.q4, c.s4);
  };
  // U^T z = gbar, local pass from a zero state with the chunk's 4x4 map
  double A[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) A[r][c] = (r == c) ? 1.0 : 0.0;
  double2 cv[4] = {zero2(), zero2(), zero2(), zero2()};
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const double r0 = R0(j);
    const double2 qs = qsj(j);
    const double e1 = -r0 * U2p(j), e2 = -r0 * U4pp(j), e3 = -r0 * qs.x, e4 = -r0 * qs.y;
    const double pp = Ppp(j), rr = Rpp(j);
    double nA0[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) nA0[c] = e1 * A[0][c] + e2 * A[1][c] + e3 * A[2][c] + e4 * A[3][c];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double a1 = A[1][c];
      A[2][c] = __builtin_fma(pp, a1, A[2][c]);
      A[3][c] = __builtin_fma(rr, a1, A[3][c]);
      A[1][c] = A[0][c];
      A[0][c] = nA0[c];
    }
    double2 nc0 = c_mul(r0, gload(grow, j));
    nc0 = c_fma(e1, cv[0], nc0);
    nc0 = c_fma(e2, cv[1], nc0);
    nc0 = c_fma(e3, cv[2], nc0);
    nc0 = c_fma(e4, cv[3], nc0);
    cv[2] = c_fma(pp, cv[1], cv[2]);
    cv[3] = c_fma(rr, cv[1], cv[3]);
    cv[1] = cv[0];
    cv[0] = nc0;
  }
  auto lvlA = [&](auto dd) {  // this chunk after the lower ones
    constexpr int D = decltype(dd)::value;
    double oA[4][4];
    double2 oc[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int c = 0; c < 4; ++c) oA[r][c] = chain_lo<G, D>(A[r][c], m);
      oc[r] = chain_lo<G, D>(cv[r], m);
    }
    double nA[4][4];
    double2 ncv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double2 acc = cv[r];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc = c_fma(A[r][c], oc[c], acc);
      ncv[r] = acc;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) t = __builtin_fma(A[r][q], oA[q][c], t);
        nA[r][c] = t;
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      cv[r] = ncv[r];
#pragma unroll
      for (int c = 0; c < 4; ++c) A[r][c] = nA[r][c];
    }
  };
  lvlA(std::integral_constant<int, 1>{});
  if constexpr (G > 2) lvlA(std::integral_constant<int, 2>{});
  if constexpr (G > 4) lvlA(std::integral_constant<int, 4>{});
  if constexpr (G > 8) lvlA(std::integral_constant<int, 8>{});
  if constexpr (G > 16) lvlA(std::integral_constant<int, 16>{});
  // incoming state from the lane below, then the exact rerun
  double2 z1 = chain_lo<G, 1>(cv[0], m), z2 = chain_lo<G, 1>(cv[1], m), SP = chain_lo<G, 1>(cv[2], m),
          SR = chain_lo<G, 1>(cv[3], m);
  uintptr_t grow_again = reinterpret_cast<uintptr_t>(grow);
  asm volatile("" : "+v"(grow_again));
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const double r0 = R0(j);
    const double2 qs = qsj(j);
    double2 z = c_mul(r0, gload(reinterpret_cast<const double2*>(grow_again), j));
    z = c_fma(-r0 * U2p(j), z1, z);
    z = c_fma(-r0 * U4pp(j), z2, z);
    z = c_fma(-r0 * qs.x, SP, z);
    z = c_fma(-r0 * qs.y, SR, z);
    SP = c_fma(Ppp(j), z2, SP);
    SR = c_fma(Rpp(j), z2, SR);
    z2 = z1;
    z1 = z;
    x[j] = z;
  }
  // L^T lambda = z: lambda_j = z_j - l1_{j+1} lambda_{j+1} - l2_{j+2} lambda_{j+2}
  const double nl1_0 = chain_hi<G, 1>(l1_0, m), nl2_0 = chain_hi<G, 1>(l2_0, m), nl2_1 = chain_hi<G, 1>(l2_1, m);
  auto L1n = [&](int j) { return j + 1 < C ? lmul[(j + 1 < C ? j + 1 : 0) * 256 + threadIdx.x].x : nl1_0; };
  auto L2nn = [&](int j) {
    return j + 2 < C ? lmul[(j + 2 < C ? j + 2 : 0) * 256 + threadIdx.x].y : (j + 2 == C ? nl2_0 : nl2_1);
  };
  double T00 = 1.0, T01 = 0.0, T10 = 0.0, T11 = 1.0;
  double2 a1v = zero2(), a2v = zero2();  // lambda_{j+1}, lambda_{j+2}
#pragma unroll
  for (int j = C - 1; j >= 0; --j) {
    const double l1 = L1n(j), l2 = L2nn(j);
    double2 v = c_fnms(l1, a1v, x[j]);
    v = c_fnms(l2, a2v, v);
    x[j] = v;
    a2v = a1v;
    a1v = v;
    const double n00 = -l1 * T00 - l2 * T10, n01 = -l1 * T01 - l2 * T11;
    T10 = T00;
    T11 = T01;
    T00 = n00;
    T01 = n01;
  }
  double2 b0 = a1v, b1 = a2v;
  auto lvlT = [&](auto dd) {  // this chunk after the upper ones
    constexpr int D = decltype(dd)::value;
    const double o00 = chain_hi<G, D>(T00, m), o01 = chain_hi<G, D>(T01, m), o10 = chain_hi<G, D>(T10, m),
                 o11 = chain_hi<G, D>(T11, m);
    const double2 ob0 = chain_hi<G, D>(b0, m), ob1 = chain_hi<G, D>(b1, m);
    const double2 n0 = c_add(c_fma(T00, ob0, c_mul(T01, ob1)), b0);
    const double2 n1 = c_add(c_fma(T10, ob0, c_mul(T11, ob1)), b1);
    const double n00 = T00 * o00 + T01 * o10, n01 = T00 * o01 + T01 * o11;
    const double n10 = T10 * o00 + T11 * o10, n11 = T10 * o01 + T11 * o11;
    T00 = n00;
    T01 = n01;
    T10 = n10;
    T11 = n11;
    b0 = n0;
    b1 = n1;
  };
  lvlT(std::integral_constant<int, 1>{});
  if constexpr (G > 2) lvlT(std::integral_constant<int, 2>{});
  if constexpr (G > 4) lvlT(std::integral_constant<int, 4>{});
  if constexpr (G > 8) lvlT(std::integral_constant<int, 8>{});
  if constexpr (G > 16) lvlT(std::integral_constant<int, 16>{});
  double2 h1 = chain_hi<G, 1>(b0, m), h2 = chain_hi<G, 1>(b1, m);  // (lambda_C, lambda_{C+1})
#pragma unroll
  for (int j = C - 1; j >= 0; --j) {
    double2 hj = c_mul(-L1n(j), h1);
    hj = c_fma(-L2nn(j), h2, hj);
    x[j] = c_add(x[j], hj);
    h2 = h1;
    h1 = hj;
  }
  if (grad_a != nullptr || grad_b != nullptr) {
    const double2* urow = ufwd + (wok ? w : 0) * (int64_t)N;
    double2 uu[C];
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int k = k0 + 2 * j;
      uu[j] = (wok && k < n) ? urow[k] : zero2();
    }
    const double2 pl1 = chain_lo<G, 1>(uu[C - 1], m), pl2 = chain_lo<G, 1>(uu[C - 2], m);
    const double2 nx1 = chain_hi<G, 1>(uu[0], m), nx2 = chain_hi<G, 1>(uu[1], m);
    double ga = 0.0, gb = 0.0;
    BihConst cm2 = bih_const_at(tab, RT, C, k0 - 2, N, gl), cm4 = bih_const_at(tab, RT, C, k0 - 4, N, gl);
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int k = k0 + 2 * j;
      const BihConst c = bih_tab_get(tab, RT, C, k);
      const double2 um4 = (j >= 2) ? uu[j >= 2 ? j - 2 : 0] : (j == 1 ? pl1 : pl2);
      const double2 um2 = (j >= 1) ? uu[j >= 1 ? j - 1 : 0] : pl1;
      const double2 up2 = (j <= C - 2) ? uu[j <= C - 2 ? j + 1 : 0] : nx1;
      const double2 up4 = (j <= C - 3) ? uu[j <= C - 3 ? j + 2 : 0] : (j == C - 2 ? nx1 : nx2);
      double2 au = c_mul(c.A0, uu[j]);
      au = c_fma(k >= 2 ? c.Am2 : 0.0, um2, au);
      au = c_fma(c.A2, up2, au);
      double2 bu = c_mul(c.B0, uu[j]);
      bu = c_fma(k >= 4 ? cm4.B4 : 0.0, um4, bu);
      bu = c_fma(k >= 2 ? cm2.B2 : 0.0, um2, bu);
      bu = c_fma(c.B2, up2, bu);
      bu = c_fma(c.B4, up4, bu);
      const bool ok = wok && k < n;
      if (ok) {
        ga -= x[j].x * au.x + x[j].y * au.y;
        gb -= x[j].x * bu.x + x[j].y * bu.y;
      }
      cm4 = cm2;
      cm2 = c;
    }
#pragma unroll
    for (int d = 1; d < 2 * G; d <<= 1) {
      ga += __shfl_xor(ga, d, 2 * G);
      gb += __shfl_xor(gb, d, 2 * G);
    }
    if (wok && (lane % (2 * G)) == 0) {
      if (grad_a) grad_a[w] = ga;
      if (grad_b) grad_b[w] = gb;
    }
  }
  if (wok) {
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int k = k0 + 2 * j;
      if (k < N) lrow[k] = (k < n) ? x[j] : zero2();
    }
  }
  if (info != nullptr) {
    int bq = bad;
#pragma unroll
    for (int d = 1; d < 2 * G; d <<= 1) bq = min(bq, __shfl_xor(bq, d, 2 * G));
    if (wok && (lane % (2 * G)) == 0) info[w] = (bq == INT_MAX) ? 0 : bq + 1;
  }
}

template <int C, int G>
__global__ __launch_bounds__(256) void bih_wave_tab(int N, int64_t nsys, const double* __restrict__ ca, const double* __restrict__ cb,
                                                    const double2* __restrict__ f, double2* __restrict__ u,
                                                    const double2* __restrict__ sts, int64_t sstride, int gl,
                                                    int32_t* __restrict__ info) {
  extern __shared__ double tab[];
  constexpr int SPW = 64 / (2 * G);
  bih_tab_fill(tab, 2 * G * C, C, N, gl, threadIdx.x, 256);
  __syncthreads();
  const int64_t wbase = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * SPW;
  bih_wave_body<C, G, true>(N, nsys, wbase, ca, cb, f, u, sts, sstride, gl, info, tab);
}

// This lane's chunk (rows k0 + 2j of system sl) and restart words from tile T.
template <int C, int G, int NS>
__device__ __forceinline__ void read_tile(const double2* T, int lane, double2 (&x)[C], double2 (&st)[NS]) {
  using TL = Tile<C, G>;
  const int sl = lane / (2 * G), p = (lane / G) & 1, m = lane % G;
  const int k0 = 2 * m * C + p;
#pragma unroll
  for (int j = 0; j < C; ++j) x[j] = T[TL::pos(sl, k0 + 2 * j)];
#pragma unroll
  for (int t = 0; t < NS; ++t) st[t] = T[64 * (C + t) + lane];
}

// As read_tile, with the LDS reads in asm that waits for them itself: used
// where stores of the previous group may still be in flight, which the
// compiler would otherwise wait for before touching a tile that an LDS-DMA
// wrote.
typedef double v2d __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void lds_read4(uint32_t a0, uint32_t a1, uint32_t a2, uint32_t a3, v2d& x0, v2d& x1, v2d& x2,
                                          v2d& x3) {
  asm volatile(
      "ds_read_b128 %0, %4\n\t"
      "ds_read_b128 %1, %5\n\t"
      "ds_read_b128 %2, %6\n\t"
      "ds_read_b128 %3, %7\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(x0), "=&v"(x1), "=&v"(x2), "=&v"(x3)
      : "v"(a0), "v"(a1), "v"(a2), "v"(a3)
      : "memory");
}
template <int C, int G, int NS>
__device__ __forceinline__ void read_tile_asm(const double2* T, int lane, double2 (&x)[C], double2 (&st)[NS]) {
  using TL = Tile<C, G>;
  static_assert(C % 4 == 0, "chunk length must be a multiple of 4");
  const int sl = lane / (2 * G), p = (lane / G) & 1, m = lane % G;
  const int k0 = 2 * m * C + p;
  const uint32_t base = (uint32_t)(uintptr_t)SHEN_LDS(T);
  double2 tmp[C + ((NS + 3) / 4) * 4];
  uint32_t ad[C + ((NS + 3) / 4) * 4];
#pragma unroll
  for (int j = 0; j < C; ++j) ad[j] = base + 16u * (uint32_t)TL::pos(sl, k0 + 2 * j);
#pragma unroll
  for (int t = 0; t < ((NS + 3) / 4) * 4; ++t) ad[C + t] = base + 16u * (uint32_t)(64 * (C + (t < NS ? t : 0)) + lane);
#pragma unroll
  for (int j = 0; j < C + ((NS + 3) / 4) * 4; j += 4) {
    v2d r0, r1, r2, r3;
    lds_read4(ad[j], ad[j + 1], ad[j + 2], ad[j + 3], r0, r1, r2, r3);
    tmp[j] = make_double2(r0.x, r0.y);
    tmp[j + 1] = make_double2(r1.x, r1.y);
    tmp[j + 2] = make_double2(r2.x, r2.y);
    tmp[j + 3] = make_double2(r3.x, r3.y);
  }
#pragma unroll
  for (int j = 0; j < C; ++j) x[j] = tmp[j];
#pragma unroll
  for (int t = 0; t < NS; ++t) st[t] = tmp[C + t];
}

// The two FP64 coefficients of each lane's system into a 1 KiB LDS area R by
// LDS-DMA (four 4-byte transfers: low and high words of a, then of b), and
// back out with asm reads.  Kept out of registers between the prefetch and
// their use, a loaded coefficient can be neither waited for early nor
// spilled (a spill would wait for every load in flight, the tile included).
__device__ __forceinline__ void prefetch_coef2(double2* R, int lane, int64_t w, const double* __restrict__ ca,
                                               const double* __restrict__ cb) {
  const int* a32 = reinterpret_cast<const int*>(ca + w);
  const int* b32 = reinterpret_cast<const int*>(cb + w);
  int* r = reinterpret_cast<int*>(R);
  __builtin_amdgcn_global_load_lds((const void*)a32, SHEN_LDS(r), 4, 0, 0);
  __builtin_amdgcn_global_load_lds((const void*)(a32 + 1), SHEN_LDS(r + 64), 4, 0, 0);
  __builtin_amdgcn_global_load_lds((const void*)b32, SHEN_LDS(r + 128), 4, 0, 0);
  __builtin_amdgcn_global_load_lds((const void*)(b32 + 1), SHEN_LDS(r + 192), 4, 0, 0);
  (void)lane;
}
__device__ __forceinline__ void read_coef2(const double2* R, int lane, double& a, double& b) {
  const uint32_t base = (uint32_t)(uintptr_t)SHEN_LDS(R) + 4u * (uint32_t)lane;
  int alo, ahi, blo, bhi;
  asm volatile(
      "ds_read_b32 %0, %4\n\t"
      "ds_read_b32 %1, %4 offset:256\n\t"
      "ds_read_b32 %2, %4 offset:512\n\t"
      "ds_read_b32 %3, %4 offset:768\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(alo), "=&v"(ahi), "=&v"(blo), "=&v"(bhi)
      : "v"(base)
      : "memory");
  a = __hiloint2double(ahi, alo);
  b = __hiloint2double(bhi, blo);
}

// Only the restart words of this lane from tile T (asm reads, as above).
template <int C, int NS>
__device__ __forceinline__ void read_states_asm(const double2* T, int lane, double2 (&st)[NS]) {
  const uint32_t base = (uint32_t)(uintptr_t)SHEN_LDS(T);
#pragma unroll
  for (int t = 0; t < NS; t += 4) {
    uint32_t ad[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) ad[q] = base + 16u * (uint32_t)(64 * (C + (t + q < NS ? t + q : 0)) + lane);
    v2d r[4];
    lds_read4(ad[0], ad[1], ad[2], ad[3], r[0], r[1], r[2], r[3]);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (t + q < NS) st[t + q] = make_double2(r[q].x, r[q].y);
  }
}

// f of chunk element j from tile T, four elements per LDS round trip (0 on
// padding rows and absent systems); serves both forward sweeps.
template <int C, int G>
struct TileFetch4 {
  static constexpr bool lazy = true;
  uint32_t base;
  int sl, k0, n;
  bool wok;
  v2d b[4];
  __device__ __forceinline__ double2 operator()(int j) {
    using TL = Tile<C, G>;
    if (j % 4 == 0) {
      uint32_t ad[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) ad[q] = base + 16u * (uint32_t)TL::pos(sl, k0 + 2 * (j + q));
      lds_read4(ad[0], ad[1], ad[2], ad[3], b[0], b[1], b[2], b[3]);
    }
    const v2d r = b[j % 4];
    return (wok && k0 + 2 * j < n) ? make_double2(r.x, r.y) : zero2();
  }
};

// Stages this lane's solution chunk in tile T.
template <int C, int G>
__device__ __forceinline__ void stage_tile(double2* T, int lane, const double2 (&x)[C]) {
  using TL = Tile<C, G>;
  const int sl = lane / (2 * G), p = (lane / G) & 1, m = lane % G;
  const int k0 = 2 * m * C + p;
#pragma unroll
  for (int j = 0; j < C; ++j) T[TL::pos(sl, k0 + 2 * j)] = x[j];
}

// Stores the staged rows k < N of group g (zero for k >= n) as whole blocks.
template <int C, int G>
__device__ __forceinline__ void store_tile(const double2* T, int lane, int64_t g, int N, int n, int64_t nsys,
                                           double2* __restrict__ u) {
  using TL = Tile<C, G>;
  double2 v[C];
#pragma unroll
  for (int i = 0; i < C; ++i) v[i] = T[64 * i + lane];
  // keep the LDS reads together (not sunk into the masked stores one by one)
  asm volatile("" ::: "memory");
#pragma unroll
  for (int i = 0; i < C; ++i) {
    const int s = i / TL::NB;
    const int64_t w = g * TL::SPW + s;
    const int k = TL::row(i, lane);
    if (w < nsys && k < N) u[w * (int64_t)N + k] = (k < n) ? v[i] : zero2();
  }
}

// Rows of sh (the scalar products S(h) of a Crank-Nicolson right-hand side)
// in store_tile's layout, 0 where there is no such row; issued before the
// tile's arithmetic, so that their latency is hidden behind it.
template <int C, int G>
__device__ __forceinline__ void load_tile_sh(int lane, int64_t g, int N, int n, int64_t nsys, const double2* __restrict__ sh,
                                             double2 (&v)[C]) {
  using TL = Tile<C, G>;
#pragma unroll
  for (int i = 0; i < C; ++i) {
    const int s = i / TL::NB;
    const int64_t w = g * TL::SPW + s;
    const int k = TL::row(i, lane);
    v[i] = (sh != nullptr && w < nsys && k < n) ? sh[w * (int64_t)N + k] : zero2();
  }
}

// As store_tile, for the Crank-Nicolson right-hand side: the staged rows hold
// -H'u, and sigma S(h) (shv from load_tile_sh) is added on the way out.
template <int C, int G>
__device__ __forceinline__ void store_tile_rhs(const double2* T, int lane, int64_t g, int N, int n, int64_t nsys,
                                               double2* __restrict__ u, double sigma, const double2 (&shv)[C]) {
  using TL = Tile<C, G>;
  double2 v[C];
#pragma unroll
  for (int i = 0; i < C; ++i) v[i] = c_fma(sigma, shv[i], T[64 * i + lane]);
  // keep the LDS reads together (not sunk into the masked stores one by one)
  asm volatile("" ::: "memory");
#pragma unroll
  for (int i = 0; i < C; ++i) {
    const int s = i / TL::NB;
    const int64_t w = g * TL::SPW + s;
    const int k = TL::row(i, lane);
    if (w < nsys && k < N) u[w * (int64_t)N + k] = (k < n) ? v[i] : zero2();
  }
}

template <int C, int G>
__global__ __launch_bounds__(64, 2) void helm_wave_pipe(int N, int64_t nsys, const double* __restrict__ alpha,
                                                     const double2* __restrict__ f, double2* __restrict__ u,
                                                     const double2* __restrict__ sts, int64_t sstride, int gl,
                                                     int32_t* __restrict__ info) {
  using TL = Tile<C, G>;
  constexpr int SPW = TL::SPW;
  __shared__ double2 tile[(C + 1) * 64];
  const int64_t ngroups = (nsys + SPW - 1) / SPW;
  const int64_t g0 = blockIdx.x;
  if (g0 >= ngroups) return;
  const int n = N - 2;
  auto coef = [&](int64_t g, int l) {
    const int64_t w = g * SPW + l / (2 * G);
    return alpha[w < nsys ? w : nsys - 1];
  };
  double2 x[C], st[1];
  double al;
  {
    const int lane = threadIdx.x & 63;
    prefetch_tile<C, G, 1>(tile, lane, g0, N, nsys, f, sts, sstride);
    al = coef(g0, lane);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    read_tile<C, G, 1>(tile, lane, x, st);
  }
  for (int64_t g = g0; g < ngroups; g += gridDim.x) {
    // Lane-derived indices are re-derived every iteration from an opaque
    // copy: hoisting the per-row constants out of the loop would hold them
    // in registers across it.
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));
  lane &= 63;  // opaque, but known to be a lane index
    const int sl = lane / (2 * G), p = (lane / G) & 1, m = lane % G;
    const int k0 = 2 * m * C + p;
    const int64_t w = g * SPW + sl;
    const bool wok = w < nsys;
#pragma unroll
    for (int j = 0; j < C; ++j) x[j] = (wok && k0 + 2 * j < n) ? x[j] : zero2();
    HelmPrev pv = {0.0, 0.0};
    if (wok && m > 0 && k0 < n) {
      pv.rd = st[0].x;
      pv.g = st[0].y;
    }
    helm_wave_core<C, G, true>(N, lane, w, wok, wok ? al : 0.0, pv, x, u, gl, info);
    stage_tile<C, G>(tile, lane, x);
    store_tile<C, G>(tile, lane, g, N, n, nsys, u);
    const int64_t gn = g + gridDim.x;
    if (gn < ngroups) {
      prefetch_tile<C, G, 1>(tile, lane, gn, N, nsys, f, sts, sstride);
      al = coef(gn, lane);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      read_tile<C, G, 1>(tile, lane, x, st);
    }
  }
}

// Persistent table-driven biharmonic wave solve: one 256-thread block per
// compute unit fills the row table once; each of its wavefronts then loops
// over groups of systems on its own, streaming the next group's right-hand
// sides and restart states into its LDS tile (whole 64-row blocks) once the
// refinement sweep has read the current group's f from it.
// Wavefronts per block of the pipelined biharmonic kernel: four for G = 16
// (two systems per wavefront, about 500 registers each: one wavefront per
// SIMD) and for C = 16, G = 32 (one system per wavefront, 1024 rows, compact
// row table); eight for C = 8, G = 32 (at most 256 registers: two per SIMD),
// all sharing one row table.
template <int C, int G>
struct PtabWaves {
  static constexpr int value = (G == 32 && C < 16) ? 8 : 4;
};

template <int C, int G>
__global__ __launch_bounds__((64 * PtabWaves<C, G>::value)) void bih_wave_ptab(int N, int64_t nsys, const double* __restrict__ ca,
                                                     const double* __restrict__ cb, const double2* __restrict__ f,
                                                     double2* __restrict__ u, const double2* __restrict__ sts,
                                                     int64_t sstride, int gl, int32_t* __restrict__ info) {
  using TL = Tile<C, G>;
  constexpr int SPW = TL::SPW;
  constexpr int RT = 2 * G * C;
  extern __shared__ double smem[];
  double* tab = smem;
  // wavefront index as a scalar: the tile base (and with it the LDS-DMA
  // destinations) and the group loop stay in scalar registers
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  double2* tile = reinterpret_cast<double2*>(smem + 2 * bih_tab_pairs(RT) * RT) + wv * ((C + 6) * 64);
  double2* coef = tile + (C + 5) * 64;  // the group's coefficients (prefetch_coef2)
  constexpr int WPB = PtabWaves<C, G>::value;
  bih_tab_fill(tab, RT, C, N, gl, threadIdx.x, 64 * WPB);
  __syncthreads();
  const int n = N - 4;
  const int64_t ngroups = (nsys + SPW - 1) / SPW;
  const int64_t stride = (int64_t)gridDim.x * WPB;
  int64_t g = (int64_t)blockIdx.x * WPB + wv;
  if (g >= ngroups) return;
  auto sysc = [&](int64_t gg, int l) {
    const int64_t w = gg * SPW + l / (2 * G);
    return w < nsys ? w : nsys - 1;
  };
  {
    const int lane = threadIdx.x & 63;
    prefetch_tile<C, G, 5>(tile, lane, g, N, nsys, f, sts, sstride);
    prefetch_coef2(coef, lane, sysc(g, lane), ca, cb);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  }
  for (; g < ngroups; g += stride) {
    // Lane-derived indices are re-derived every iteration from an opaque
    // copy: hoisting the per-row constants out of the loop would hold them
    // in registers across it.
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));
    lane &= 63;  // opaque, but known to be a lane index
    const int sl = lane / (2 * G), p = (lane / G) & 1, m = lane % G;
    const int k0 = 2 * m * C + p;
    const int64_t w = g * SPW + sl;
    const bool wok = w < nsys;
    double2 x[C], st[5];
    read_states_asm<C, 5>(tile, lane, st);  // f is read by the sweeps themselves
    double ca_, cb_;
    read_coef2(coef, lane, ca_, cb_);
    BihRowState m2 = {0, 0, 0, 0, 0}, m4 = {0, 0, 0, 0, 0};
    if (wok && m > 0 && k0 < n) {
      m2 = BihRowState{st[0].x, st[0].y, st[1].x, st[1].y, st[2].x};
      m4 = BihRowState{st[2].y, st[3].x, st[3].y, st[4].x, st[4].y};
    }
    TileFetch4<C, G> fetch;
    fetch.base = (uint32_t)(uintptr_t)SHEN_LDS(tile);
    fetch.sl = sl;
    fetch.k0 = k0;
    fetch.n = n;
    fetch.wok = wok;
    const int64_t gn = g + stride;
    auto prefetch_next = [&]() {
      if (gn < ngroups) {
        prefetch_tile<C, G, 5>(tile, lane, gn, N, nsys, f, sts, sstride);
        prefetch_coef2(coef, lane, sysc(gn, lane), ca, cb);
      }
    };
    double2* urow = u + (wok ? w : 0) * (int64_t)N;
    bih_wave_core<C, G, true, true>(N, lane, w, wok, wok ? ca_ : 0.0, wok ? cb_ : 0.0, m2, m4, x, fetch, urow, gl, info, tab,
                                    prefetch_next, std::true_type{}, walk_bad_of(st[0].x, wok && m == 0));
    // The next group has landed.  This group's solution is stored only after
    // this wait, so that the wait does not include the acknowledgement of
    // its stores; they complete while the next group is solved.
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    if (wok) {
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const int k = k0 + 2 * j;
        if (k < N) urow[k] = x[j];  // table rows past n solve to zero
      }
    }
  }
}


// =========================================================================
// Matrix-vector products H u in the wave layout (right-hand-side assembly and
// residuals, Sec. 3): persistent kernels that stream each group's u into an
// LDS tile, take it into registers, form H u from each lane's chunk and its
// neighbours (helm_apply / bih_apply), and send it out through the same tile
// as whole 64-row blocks before the next group's tile comes in.  Rows
// k >= n are written as 0.
// =========================================================================
template <int C, int G>
__device__ __forceinline__ void read_tile_rows(const double2* T, int lane, int n, bool wok, double2 (&x)[C]) {
  using TL = Tile<C, G>;
  const int sl = lane / (2 * G), p = (lane / G) & 1, m = lane % G;
  const int k0 = 2 * m * C + p;
  const uint32_t base = (uint32_t)(uintptr_t)SHEN_LDS(T);
#pragma unroll
  for (int j = 0; j < C; j += 4) {
    v2d r[4];
    lds_read4(base + 16u * (uint32_t)TL::pos(sl, k0 + 2 * j), base + 16u * (uint32_t)TL::pos(sl, k0 + 2 * j + 2),
              base + 16u * (uint32_t)TL::pos(sl, k0 + 2 * j + 4), base + 16u * (uint32_t)TL::pos(sl, k0 + 2 * j + 6), r[0],
              r[1], r[2], r[3]);
#pragma unroll
    for (int q = 0; q < 4; ++q) x[j + q] = (wok && k0 + 2 * (j + q) < n) ? make_double2(r[q].x, r[q].y) : zero2();
  }
}

// RHS: alpha holds K2 per system, and the kernel writes the Crank-Nicolson
// right-hand side sigma S(h) - (S + alpha' B) u, alpha' = K2 - inv (sh = S(h)
// rows, or null), instead of H u.
template <int C, int G, bool RHS = false>
__global__ __launch_bounds__(64) void helm_matvec_pipe(int N, int64_t nsys, const double* __restrict__ alpha,
                                                       const double2* __restrict__ uin, double2* __restrict__ hu, int gl,
                                                       double inv = 0.0, double sigma = 0.0,
                                                       const double2* __restrict__ sh = nullptr) {
  using TL = Tile<C, G>;
  constexpr int SPW = TL::SPW;
  __shared__ double2 tile[(C + 1) * 64];
  double2* coef = tile + C * 64;
  const int64_t ngroups = (nsys + SPW - 1) / SPW;
  int64_t g = blockIdx.x;
  if (g >= ngroups) return;
  const int n = N - 2;
  auto sysc = [&](int64_t gg, int l) {
    const int64_t w = gg * SPW + l / (2 * G);
    return w < nsys ? w : nsys - 1;
  };
  {
    const int lane = threadIdx.x & 63;
    prefetch_tile<C, G, 0>(tile, lane, g, N, nsys, uin, nullptr, 0);
    prefetch_coef2(coef, lane, sysc(g, lane), alpha, alpha);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  }
  for (; g < ngroups; g += gridDim.x) {
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));
    lane &= 63;  // opaque, but known to be a lane index
    const int64_t w = g * SPW + lane / (2 * G);
    const bool wok = w < nsys;
    double2 x[C], y[C];
    read_tile_rows<C, G>(tile, lane, n, wok, x);
    double al, unused;
    read_coef2(coef, lane, al, unused);
    double2 shv[RHS ? C : 1];
    if constexpr (RHS) {
      al = rhs_alpha(al, inv);
      load_tile_sh<C, G>(lane, g, N, n, nsys, sh, shv);
    }
    helm_apply<C, G>(N, lane, al, gl, x, [&](int j, double2 v) { y[j] = RHS ? make_double2(-v.x, -v.y) : v; });
    stage_tile<C, G>(tile, lane, y);
    if constexpr (RHS) {
      store_tile_rhs<C, G>(tile, lane, g, N, n, nsys, hu, sigma, shv);
    } else {
      store_tile<C, G>(tile, lane, g, N, n, nsys, hu);
    }
    const int64_t gn = g + gridDim.x;
    if (gn < ngroups) {
      prefetch_tile<C, G, 0>(tile, lane, gn, N, nsys, uin, nullptr, 0);
      prefetch_coef2(coef, lane, sysc(gn, lane), alpha, alpha);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
  }
}

// RHS: ca holds K2 per system, and the kernel writes the Crank-Nicolson
// right-hand side sigma S(h) - (Q + a' A + b' B) u, a' = inv - 2 K2,
// b' = K2 (K2 - inv) (sh = S(h) rows, or null), instead of H u.
template <int C, int G, bool RHS = false>
__global__ __launch_bounds__(256) void bih_matvec_ptab(int N, int64_t nsys, const double* __restrict__ ca,
                                                       const double* __restrict__ cb, const double2* __restrict__ uin,
                                                       double2* __restrict__ hu, int gl, double inv = 0.0, double sigma = 0.0,
                                                       const double2* __restrict__ sh = nullptr) {
  using TL = Tile<C, G>;
  constexpr int SPW = TL::SPW;
  constexpr int RT = 2 * G * C;
  extern __shared__ double smem[];
  double* tab = smem;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  double2* tile = reinterpret_cast<double2*>(smem + 2 * bih_tab_pairs(RT) * RT) + wv * ((C + 1) * 64);
  double2* coef = tile + C * 64;
  bih_tab_fill(tab, RT, C, N, gl, threadIdx.x, 256);
  __syncthreads();
  const int n = N - 4;
  const int64_t ngroups = (nsys + SPW - 1) / SPW;
  const int64_t stride = (int64_t)gridDim.x * 4;
  int64_t g = (int64_t)blockIdx.x * 4 + wv;
  if (g >= ngroups) return;
  auto sysc = [&](int64_t gg, int l) {
    const int64_t w = gg * SPW + l / (2 * G);
    return w < nsys ? w : nsys - 1;
  };
  {
    const int lane = threadIdx.x & 63;
    prefetch_tile<C, G, 0>(tile, lane, g, N, nsys, uin, nullptr, 0);
    prefetch_coef2(coef, lane, sysc(g, lane), ca, cb);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  }
  for (; g < ngroups; g += stride) {
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));
    lane &= 63;  // opaque, but known to be a lane index
    const int64_t w = g * SPW + lane / (2 * G);
    const bool wok = w < nsys;
    double2 x[C], y[C];
    read_tile_rows<C, G>(tile, lane, n, wok, x);
    double a, b;
    read_coef2(coef, lane, a, b);
    double2 shv[RHS ? C : 1];
    if constexpr (RHS) {
      const double K2 = a;
      a = rhs_a(K2, inv);
      b = rhs_b(K2, inv);
      load_tile_sh<C, G>(lane, g, N, n, nsys, sh, shv);
    }
    bih_apply<C, G>(N, lane, a, b, gl, tab, x, [&](int j, double2 v) { y[j] = RHS ? make_double2(-v.x, -v.y) : v; });
    stage_tile<C, G>(tile, lane, y);
    if constexpr (RHS) {
      store_tile_rhs<C, G>(tile, lane, g, N, n, nsys, hu, sigma, shv);
    } else {
      store_tile<C, G>(tile, lane, g, N, n, nsys, hu);
    }
    const int64_t gn = g + stride;
    if (gn < ngroups) {
      prefetch_tile<C, G, 0>(tile, lane, gn, N, nsys, uin, nullptr, 0);
      prefetch_coef2(coef, lane, sysc(gn, lane), ca, cb);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
  }
}

// =========================================================================
// Mass-matrix solves u = B^{-1} f (the last step of a forward Shen transform,
// Sec. 2: u_hat = B^{-1} S(u)).  One matrix serves every system: Bbar
// (Dirichlet basis, FAM 0) couples rows k-2, k, k+2, and Bchk (biharmonic
// basis, FAM 1) rows k-4 .. k+4, so per parity chain they are tri- and
// pentadiagonal, with bandwidth S = 1 or 2 in chain index.
//
// Each work group factors both chains once (no pivoting: B is symmetric
// positive definite) into an LDS table, and each lane keeps the factors of
// its chunk in registers for the whole persistent loop.  Per group of systems
// the forward and backward recurrences run as in the solves: a chunk sweep
// from a zero state gives the chunk's affine map on the S-vector state (its
// matrix depends on the factors only and is formed once per lane), a
// Kogge-Stone scan over the chain's lanes combines the maps, and each lane
// reruns its chunk from the scanned incoming state.  Rows k >= n are
// identity rows with zero right-hand side, so they solve to zero unmasked.
// =========================================================================
template <int FAM>
struct MassFields {
  static constexpr int S = FAM == 0 ? 1 : 2;
  static constexpr int NF = 2 * S + 1;  // l_1..l_S, 1/U0, U_1..U_S
};

// Band entries of rows k < RT into the table [NF][RT] (row slots swizzled
// like the biharmonic row table), fields e_{-S} .. e_{-1}, e_0, e_{+1} ..
// e_{+S} in chain offsets.  Rows k >= n are identity rows, and the couplings
// of the last rows to columns >= n are dropped.
template <int FAM>
__device__ __forceinline__ void mass_entries_fill(double* tab, int RT, int C, int N, int gl, int tid, int nthreads) {
  const int n = FAM == 0 ? N - 2 : N - 4;
  for (int k = tid; k < RT; k += nthreads) {
    const int r = bih_tab_row(k, C);
    if constexpr (FAM == 0) {
      const bool in = k < n;
      tab[0 * RT + r] = in && k >= 2 ? -0.5 * kPi : 0.0;
      tab[1 * RT + r] = in ? helm_mass_diag(k, N, gl) : 1.0;
      tab[2 * RT + r] = in && k + 2 < n ? -0.5 * kPi : 0.0;
    } else {
      double e[5] = {0.0, 0.0, 1.0, 0.0, 0.0};
      if (k < n) {
        // B is ill-conditioned, so its entries are formed with IEEE divisions
        // (a one-time cost per work group) rather than refined estimates.
        const double K = (double)k;
        Recip R;
        R.m1 = k == 1 ? 0.0 : 1.0 / (K - 1.0);
        R.p1 = 1.0 / (K + 1.0);
        R.p3 = 1.0 / (K + 3.0);
        R.p5 = 1.0 / (K + 5.0);
        R.p7 = 1.0 / (K + 7.0);
        const BihMats mm = bih_mats(k, N, gl, R);
        e[0] = mm.Bm4;
        e[1] = mm.Bm2;
        e[2] = mm.B0;
        e[3] = k + 2 < n ? mm.B2 : 0.0;
        e[4] = k + 4 < n ? mm.B4 : 0.0;
      }
#pragma unroll
      for (int t = 0; t < 5; ++t) tab[t * RT + r] = e[t];
    }
  }
}

// Sequential banded LU (no pivoting) of chain p, rows k = p, p+2, ... < RT,
// in place over the band entries: fields l_1..l_S (multipliers of rows
// i-1..i-S), 1/U0, U_1..U_S (the upper band of row i).
template <int FAM>
__device__ __forceinline__ void mass_lu_chain(double* tab, int RT, int C, int p) {
  constexpr int S = MassFields<FAM>::S;
  double rdp[2] = {0.0, 0.0}, U1p[2] = {0.0, 0.0}, U2p[2] = {0.0, 0.0};  // index 0: row i-1
  for (int k = p; k < RT; k += 2) {
    const int r = bih_tab_row(k, C);
    double e2 = 0.0, u2 = 0.0;
    if constexpr (S == 2) {
      e2 = tab[0 * RT + r];
      u2 = tab[4 * RT + r];
    }
    const double e1 = tab[(S - 1) * RT + r], e0 = tab[S * RT + r], u1 = tab[(S + 1) * RT + r];
    double l2 = 0.0, t1 = e1, t0 = e0;
    if constexpr (S == 2) {
      l2 = e2 * rdp[1];
      t1 = __builtin_fma(-l2, U1p[1], t1);
      t0 = __builtin_fma(-l2, U2p[1], t0);
    }
    const double l1 = t1 * rdp[0];
    t0 = __builtin_fma(-l1, U1p[0], t0);
    const double U1 = S == 2 ? __builtin_fma(-l1, U2p[0], u1) : u1;
    const double rd = 1.0 / t0;
    tab[0 * RT + r] = l1;
    if constexpr (S == 2) tab[1 * RT + r] = l2;
    tab[S * RT + r] = rd;
    tab[(S + 1) * RT + r] = U1;
    if constexpr (S == 2) tab[(S + 2) * RT + r] = u2;
    rdp[1] = rdp[0];
    U1p[1] = U1p[0];
    U2p[1] = U2p[0];
    rdp[0] = rd;
    U1p[0] = U1;
    U2p[0] = u2;
  }
}

// Affine map on an S-vector of complex states: s -> A s + c.
template <int S>
struct MassMap {
  double A[S][S];
  double2 c[S];
};

template <int S>
__device__ __forceinline__ void mass_compose(MassMap<S>& m, const MassMap<S>& q) {  // m <- m o q
  double2 c[S];
  double A[S][S];
#pragma unroll
  for (int i = 0; i < S; ++i) {
    c[i] = m.c[i];
#pragma unroll
    for (int t = 0; t < S; ++t) {
      c[i].x = __builtin_fma(m.A[i][t], q.c[t].x, c[i].x);
      c[i].y = __builtin_fma(m.A[i][t], q.c[t].y, c[i].y);
    }
#pragma unroll
    for (int j = 0; j < S; ++j) {
      double a = 0.0;
#pragma unroll
      for (int t = 0; t < S; ++t) a = __builtin_fma(m.A[i][t], q.A[t][j], a);
      A[i][j] = a;
    }
  }
#pragma unroll
  for (int i = 0; i < S; ++i) {
    m.c[i] = c[i];
#pragma unroll
    for (int j = 0; j < S; ++j) m.A[i][j] = A[i][j];
  }
}

// Inclusive scan of the chunk maps over the G lanes of a chain, towards
// higher lanes (UP = false: partner m - D, the forward recurrence) or lower
// ones (UP = true: partner m + D, the backward one); a partner past the chain
// end arrives as the zero map, which leaves the offset unchanged.
template <int G, int S, bool UP, int D>
__device__ __forceinline__ void mass_scan_steps(int m, MassMap<S>& mp) {
  if constexpr (D < G) {
    MassMap<S> q;
#pragma unroll
    for (int i = 0; i < S; ++i) {
      q.c[i] = UP ? chain_hi<G, D>(mp.c[i], m) : chain_lo<G, D>(mp.c[i], m);
#pragma unroll
      for (int j = 0; j < S; ++j) q.A[i][j] = UP ? chain_hi<G, D>(mp.A[i][j], m) : chain_lo<G, D>(mp.A[i][j], m);
    }
    mass_compose<S>(mp, q);
    mass_scan_steps<G, S, UP, 2 * D>(m, mp);
  }
}
// Incoming state of this lane's chunk: the combined map of the chunks before
// it (in the direction of the recurrence) applied to a zero state.
template <int G, int S, bool UP>
__device__ __forceinline__ void mass_scan(int m, MassMap<S> mp, double2 (&sin)[S]) {
  mass_scan_steps<G, S, UP, 1>(m, mp);
#pragma unroll
  for (int i = 0; i < S; ++i) sin[i] = UP ? chain_hi<G, 1>(mp.c[i], m) : chain_lo<G, 1>(mp.c[i], m);
}

// Rows of Cbar = (phichk_j', phibar_k)_sigma (appendix matrix table): Dirichlet
// row k couples the biharmonic coefficients j = k-3, k-1, k+1 of the other
// parity, with entries pi (k-2)(k+1)/k, -2 pi (k+1)^2/(k+2) and pi (k+1).
// Tabulated per row k < RT (zero outside rows < N-2 and columns < N-4), in
// three fields swizzled like the factor table.
__device__ __forceinline__ void deriv_entries_fill(double* ct, int RT, int C, int N, int tid, int nthreads) {
  const int nd = N - 2, nb = N - 4;
  for (int k = tid; k < RT; k += nthreads) {
    const int r = bih_tab_row(k, C);
    const double K = (double)k;
    const bool row = k < nd;
    ct[0 * RT + r] = row && k >= 3 ? kPi * (K - 2.0) * (K + 1.0) / K : 0.0;
    ct[1 * RT + r] = row && k >= 1 && k - 1 < nb ? -2.0 * kPi * (K + 1.0) * (K + 1.0) / (K + 2.0) : 0.0;
    ct[2 * RT + r] = row && k + 1 < nb ? kPi * (K + 1.0) : 0.0;
  }
}

// x_j = (Cbar uhat)_k for this lane's rows k = k0 + 2j, uhat read from the
// group's tile at rows of the other parity (selected to zero outside 0 .. N-5,
// so that whatever the ignored entries hold never enters).
template <int C, int G>
__device__ __forceinline__ void deriv_rows(const double2* T, const double* ct, int RT, int lane, int N, bool wok,
                                           double2 (&x)[C]) {
  using TL = Tile<C, G>;
  const int sl = lane / (2 * G), p = (lane / G) & 1, m = lane % G;
  const int k0 = 2 * m * C + p;
  const int nb = N - 4;
  auto U = [&](int j) {
    const bool in = j >= 0 && j < nb;
    const double2 v = T[TL::pos(sl, in ? j : 0)];  // rows past 2GC lie outside the tile
    return in ? v : zero2();
  };
  double2 um3 = U(k0 - 3), um1 = U(k0 - 1);
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int k = k0 + 2 * j;
    const int r = bih_tab_row(k, C);
    const double2 up1 = U(k + 1);
    const double c3 = ct[0 * RT + r], c1 = ct[1 * RT + r], cp = ct[2 * RT + r];
    double2 v;
    v.x = __builtin_fma(c3, um3.x, __builtin_fma(c1, um1.x, cp * up1.x));
    v.y = __builtin_fma(c3, um3.y, __builtin_fma(c1, um1.y, cp * up1.y));
    x[j] = wok ? v : zero2();
    um3 = um1;
    um1 = up1;
  }
}

// Derivative right-hand side (OP = 1): the three entries of row k of Cbar,
// at columns k-3, k-1, k+1, follow the factors in the table.
template <int C, int G, int FAM, int OP = 0>
struct MassLds {
  static constexpr int RT = 2 * G * C;
  static constexpr int NT = MassFields<FAM>::NF + (OP ? 3 : 0);  // table fields
  static constexpr size_t tab = (size_t)NT * RT * sizeof(double);
  static constexpr size_t tile = (size_t)C * 64 * sizeof(double2);
  // wavefronts per work group: eight tiles where they fit the 160 KiB, else four
  static constexpr int WPB = tab + 8 * tile <= 160 * 1024 ? 8 : 4;
  static constexpr size_t bytes = tab + WPB * tile;
};

template <int C, int G, int FAM, int OP>
__global__ __launch_bounds__((64 * MassLds<C, G, FAM, OP>::WPB)) void mass_wave_pipe(int N, int64_t nsys,
                                                                                     const double2* __restrict__ f,
                                                                                     double2* __restrict__ u, int gl) {
  static_assert(OP == 0 || FAM == 0, "the derivative right-hand side belongs to the Dirichlet solve");
  using TL = Tile<C, G>;
  using L = MassLds<C, G, FAM, OP>;
  constexpr int SPW = TL::SPW;
  constexpr int S = MassFields<FAM>::S;
  constexpr int RT = L::RT;
  extern __shared__ double smem[];
  double* tab = smem;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  double2* tile = reinterpret_cast<double2*>(smem + L::NT * RT) + wv * (C * 64);
  mass_entries_fill<FAM>(tab, RT, C, N, gl, (int)threadIdx.x, (int)blockDim.x);
  if constexpr (OP == 1) deriv_entries_fill(tab + MassFields<FAM>::NF * RT, RT, C, N, (int)threadIdx.x, (int)blockDim.x);
  __syncthreads();
  if (threadIdx.x < 2) mass_lu_chain<FAM>(tab, RT, C, (int)threadIdx.x);
  const int n = FAM == 0 ? N - 2 : N - 4;
  const int64_t ngroups = (nsys + SPW - 1) / SPW;
  const int64_t stride = (int64_t)gridDim.x * L::WPB;
  int64_t g = (int64_t)blockIdx.x * L::WPB + wv;
  const int lane = threadIdx.x & 63;
  if (g < ngroups) prefetch_tile<C, G, 0>(tile, lane, g, N, nsys, f, nullptr, 0);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (g >= ngroups) return;
  const int p = (lane / G) & 1, m = lane % G;
  const int k0 = 2 * m * C + p;
  // This lane's factors stay in registers for the whole loop where they are
  // few enough; otherwise (the pentadiagonal factors of 16-row chunks) every
  // sweep reads them from the table, which keeps the kernel at two
  // wavefronts per SIMD without spills.
  constexpr bool kRegF = MassFields<FAM>::NF * C <= 48;
  constexpr int CR = kRegF ? C : 1;
  double lf[S][CR], rd[CR], uf[S][CR];
  if constexpr (kRegF) {
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int r = bih_tab_row(k0 + 2 * j, C);
#pragma unroll
      for (int t = 0; t < S; ++t) {
        lf[t][j] = tab[t * RT + r];
        uf[t][j] = tab[(S + 1 + t) * RT + r];
      }
      rd[j] = tab[S * RT + r];
    }
  }
  // factor accessors for the lane whose first row is kb
  auto LF = [&](int kb, int t, int j) -> double {
    if constexpr (kRegF) return lf[t][j];
    else return tab[t * RT + bih_tab_row(kb + 2 * j, C)];
  };
  auto UF = [&](int kb, int t, int j) -> double {
    if constexpr (kRegF) return uf[t][j];
    else return tab[(S + 1 + t) * RT + bih_tab_row(kb + 2 * j, C)];
  };
  auto RD = [&](int kb, int j) -> double {
    if constexpr (kRegF) return rd[j];
    else return tab[S * RT + bih_tab_row(kb + 2 * j, C)];
  };
  // the homogeneous parts of this lane's chunk maps
  MassMap<S> fw, bw;  // A parts: state of the last (first) rows from the incoming state
#pragma unroll
  for (int b = 0; b < S; ++b) {
    double st[S];
#pragma unroll
    for (int t = 0; t < S; ++t) st[t] = t == b ? 1.0 : 0.0;
#pragma unroll
    for (int j = 0; j < C; ++j) {
      double y = 0.0;
#pragma unroll
      for (int t = 0; t < S; ++t) y = __builtin_fma(-LF(k0, t, j), st[t], y);
#pragma unroll
      for (int t = S - 1; t > 0; --t) st[t] = st[t - 1];
      st[0] = y;
    }
#pragma unroll
    for (int t = 0; t < S; ++t) fw.A[t][b] = st[t];
#pragma unroll
    for (int t = 0; t < S; ++t) st[t] = t == b ? 1.0 : 0.0;
#pragma unroll
    for (int j = C - 1; j >= 0; --j) {
      double v = 0.0;
#pragma unroll
      for (int t = 0; t < S; ++t) v = __builtin_fma(-UF(k0, t, j), st[t], v);
      v *= RD(k0, j);
#pragma unroll
      for (int t = S - 1; t > 0; --t) st[t] = st[t - 1];
      st[0] = v;
    }
#pragma unroll
    for (int t = 0; t < S; ++t) bw.A[t][b] = st[t];
  }
  for (; g < ngroups; g += stride) {
    // tile indices are re-derived every iteration from an opaque copy of the
    // lane (hoisted out of the loop they would hold registers across it)
    int ln = threadIdx.x & 63;
    asm volatile("" : "+v"(ln));
    ln &= 63;
    const int64_t w = g * SPW + ln / (2 * G);
    const bool wok = w < nsys;
    const int kl = 2 * (ln % G) * C + ((ln / G) & 1);
    // without register-resident factors, each sweep reads its own (no value
    // is kept live from one sweep to the next)
    auto sweep_fence = [&]() {
      if constexpr (!kRegF) asm volatile("" ::: "memory");
    };
    double2 x[C];
    if constexpr (OP == 0)
      read_tile_rows<C, G>(tile, ln, n, wok, x);
    else
      deriv_rows<C, G>(tile, tab + MassFields<FAM>::NF * RT, RT, ln, N, wok, x);
    // forward: y_i = x_i - sum_t l_t y_{i-1-t}; state (y_{i-1}, .., y_{i-S})
    double2 st[S], sin[S];
#pragma unroll
    for (int t = 0; t < S; ++t) st[t] = zero2();
#pragma unroll
    for (int j = 0; j < C; ++j) {
      double2 y = x[j];
#pragma unroll
      for (int t = 0; t < S; ++t) {
        const double l = LF(kl, t, j);
        y.x = __builtin_fma(-l, st[t].x, y.x);
        y.y = __builtin_fma(-l, st[t].y, y.y);
      }
#pragma unroll
      for (int t = S - 1; t > 0; --t) st[t] = st[t - 1];
      st[0] = y;
    }
#pragma unroll
    for (int t = 0; t < S; ++t) fw.c[t] = st[t];
    mass_scan<G, S, false>(m, fw, sin);
    sweep_fence();
#pragma unroll
    for (int t = 0; t < S; ++t) st[t] = sin[t];
#pragma unroll
    for (int j = 0; j < C; ++j) {
      double2 y = x[j];
#pragma unroll
      for (int t = 0; t < S; ++t) {
        const double l = LF(kl, t, j);
        y.x = __builtin_fma(-l, st[t].x, y.x);
        y.y = __builtin_fma(-l, st[t].y, y.y);
      }
#pragma unroll
      for (int t = S - 1; t > 0; --t) st[t] = st[t - 1];
      st[0] = y;
      x[j] = y;
    }
    sweep_fence();
    // backward: u_i = (y_i - sum_t U_t u_{i+1+t}) / U0; state (u_{i+1}, .., u_{i+S})
#pragma unroll
    for (int t = 0; t < S; ++t) st[t] = zero2();
#pragma unroll
    for (int j = C - 1; j >= 0; --j) {
      double2 v = x[j];
#pragma unroll
      for (int t = 0; t < S; ++t) {
        const double uu = UF(kl, t, j);
        v.x = __builtin_fma(-uu, st[t].x, v.x);
        v.y = __builtin_fma(-uu, st[t].y, v.y);
      }
      const double r = RD(kl, j);
      v.x *= r;
      v.y *= r;
#pragma unroll
      for (int t = S - 1; t > 0; --t) st[t] = st[t - 1];
      st[0] = v;
    }
#pragma unroll
    for (int t = 0; t < S; ++t) bw.c[t] = st[t];
    mass_scan<G, S, true>(m, bw, sin);
    sweep_fence();
#pragma unroll
    for (int t = 0; t < S; ++t) st[t] = sin[t];
#pragma unroll
    for (int j = C - 1; j >= 0; --j) {
      double2 v = x[j];
#pragma unroll
      for (int t = 0; t < S; ++t) {
        const double uu = UF(kl, t, j);
        v.x = __builtin_fma(-uu, st[t].x, v.x);
        v.y = __builtin_fma(-uu, st[t].y, v.y);
      }
      const double r = RD(kl, j);
      v.x *= r;
      v.y *= r;
#pragma unroll
      for (int t = S - 1; t > 0; --t) st[t] = st[t - 1];
      st[0] = v;
      x[j] = v;
    }
    // out through the tile as whole 64-row blocks, then the next group in
    stage_tile<C, G>(tile, ln, x);
    store_tile<C, G>(tile, ln, g, N, n, nsys, u);
    const int64_t gn = g + stride;
    if (gn < ngroups) {
      prefetch_tile<C, G, 0>(tile, ln, gn, N, nsys, f, nullptr, 0);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
  }
}

// =========================================================================
// Large N: chains longer than one wavefront, C = 16, G = 32 (512 chain
// elements per G-lane group), the wave cores with cross-wavefront carries.
// Two layouts:
//  * up to 2048 elements per chain (N <= 4096): one system per work group of
//    W wavefronts, both parity chains in every wavefront (WaveCarry);
//  * up to 4096 (N <= 8192): one parity chain per work group of W
//    wavefronts, whose 2W half-wavefronts are consecutive segments of it
//    (ChainCarry); the two chains of a system solve in different work groups.
// The boundary walk runs one thread per chain over the whole chain and parks
// the restart state of every chunk in the output row: with two parities per
// work group at [(p Gt + c) s + i] (s = 1 or 5 double2 per state, Gt chunks
// per chain); with one parity per work group interleaved by parity, at
// [2 (c s + i) + p], so that neither chain's solve writes (rows of its own
// parity) where the other still reads its states.  In that layout the walk
// also makes the pivot checks of every row (it runs the same factorisation)
// and writes info.  Both walk and solve compute the row entries (no table,
// which would not fit in LDS), so the stitched factors are bitwise those of
// the sequential LU.
// =========================================================================
static constexpr int kMultiC = 16, kMultiG = 32;

// Helmholtz walk over one chain, a chunk of C rows at a time (unrolled, so
// that the entries of later rows are formed while the recurrence of earlier
// ones runs; one wavefront per SIMD leaves that latency exposed otherwise),
// parking the state entering every later chunk: interleaved by parity (IL,
// double2 slot 2c + p) or at slot p Gt + c.  CHECK: step through the whole
// chain and return its first unusable row (INT_MAX: none); else stop at the
// last chunk start.
template <int C, bool IL, bool CHECK>
__device__ __forceinline__ int helm_walk_chain(int N, int Gt, int p, double al, double2* __restrict__ urow, int gl) {
  const int n = N - 2;
  const int nc = (n - p + 1) / 2;
  const int nchunks = (nc + C - 1) / C;
  const int cend = CHECK ? nchunks : nchunks - 1;
  HelmPrev pv = {0.0, 0.0};
  int bad = INT_MAX;
  for (int c = 0; c < cend; ++c) {
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int i = c * C + j;
      const int k = 2 * i + p;
      double l, g, rd, d, sc;
      helm_step(k, al, N, gl, pv, l, g, rd, d, sc);
      if constexpr (CHECK) bad = first_bad(bad, i < nc && bad_pivot(d, sc), k);
      pv.rd = rd;
      pv.g = g;
    }
    if (c + 1 < nchunks) urow[IL ? 2 * (c + 1) + p : p * Gt + c + 1] = make_double2(pv.rd, pv.g);
  }
  return bad;
}

// Lowest bad row of the two chains of system w (threads t and t ^ 1) -> info[w].
__device__ __forceinline__ void walk_info(int bad, bool act, int p, int64_t w, int32_t* __restrict__ info) {
  bad = min(bad, __shfl_xor(bad, 1));
  if (act && p == 0) info[w] = (bad == INT_MAX) ? 0 : bad + 1;
}

// The first unusable row of a chain (-1: none), parked by a factor call of the
// one-parity layout in the slot its chain leaves unused (chunk 0), where the
// factored solve reads it back for info.
__device__ __forceinline__ void park_bad(double2* __restrict__ srow, int p, int bad) {
  srow[p] = make_double2(bad == INT_MAX ? -1.0 : (double)bad, 0.0);
}
__device__ __forceinline__ int parked_bad(const double2* __restrict__ srow, int p) {
  const double v = srow[p].x;
  return v >= 0.0 ? (int)v : INT_MAX;
}

// States of system w go to S + w sstride (the output row, or a factor buffer).
// ONE: the interleaved layout; CHECK: the pivot checks of every row, for info
// (one-call solves) or the parked first bad rows (factor calls).
template <bool ONE, bool CHECK = ONE>
__global__ __launch_bounds__(256) void helm_walk_multi(int N, int64_t nsys, int Gt, const double* __restrict__ alpha,
                                                       double2* __restrict__ S, int64_t sstride, int gl,
                                                       int32_t* __restrict__ info, int park) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = t < 2 * nsys;  // both threads of a system share this (2 nsys is even)
  if (!act) return;
  const int64_t w = t >> 1;
  const int p = (int)(t & 1);
  double2* srow = S + w * sstride;
  const int bad = helm_walk_chain<kMultiC, ONE, CHECK>(N, Gt, p, alpha[w], srow, gl);
  if constexpr (CHECK) {
    if (info != nullptr) walk_info(bad, act, p, w, info);
    if (park) park_bad(srow, p, bad);
  }
}

// The biharmonic walk over whole chains: every thread of a block walks the
// same rows (its parity's), so the coefficient-free entries of the next
// 2 kWalkWin rows (bih_mats, the values the solve computes for the same rows)
// are formed once per block into an LDS window, and each thread only combines
// them with its coefficients (bih_row_from) before the factorisation step.
static constexpr int kWalkWin = 64;      // chain elements per window
static constexpr int kWalkWords = 18;    // doubles per window row (17 used)
__device__ __forceinline__ void mats_put(double* d, const BihMats& m) {
  d[0] = m.Bm4, d[1] = m.Am2, d[2] = m.Bm2, d[3] = m.Q0, d[4] = m.A0, d[5] = m.B0, d[6] = m.Q2, d[7] = m.A2, d[8] = m.B2;
  d[9] = m.Q4, d[10] = m.B4, d[11] = m.p, d[12] = m.r, d[13] = m.q2, d[14] = m.s2, d[15] = m.q4, d[16] = m.s4;
}
__device__ __forceinline__ BihMats mats_get(const double* d) {
  BihMats m;
  m.Bm4 = d[0], m.Am2 = d[1], m.Bm2 = d[2], m.Q0 = d[3], m.A0 = d[4], m.B0 = d[5], m.Q2 = d[6], m.A2 = d[7], m.B2 = d[8];
  m.Q4 = d[9], m.B4 = d[10], m.p = d[11], m.r = d[12], m.q2 = d[13], m.s2 = d[14], m.q4 = d[15], m.s4 = d[16];
  return m;
}
template <bool ONE, bool CHECK = ONE>
__global__ __launch_bounds__(256) void bih_walk_multi(int N, int64_t nsys, int Gt, const double* __restrict__ ca,
                                                      const double* __restrict__ cb, double2* __restrict__ S,
                                                      int64_t sstride, int gl, int32_t* __restrict__ info, int park) {
  constexpr int C = kMultiC;
  __shared__ double win[2 * kWalkWin * kWalkWords];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = t < 2 * nsys;  // inactive threads still take part in the barriers
  const int64_t w = act ? t >> 1 : 0;
  const int p = (int)(t & 1);
  const int n = N - 4;
  const int nc = (n - p + 1) / 2;
  const int nch = (nc + C - 1) / C;              // chunks of this chain
  const int nch0 = ((n + 1) / 2 + C - 1) / C;    // of the longest chain (p = 0)
  // chunks stepped through by the block: up to the last chunk start, or
  // (checking every pivot) the whole chain
  const int cend = CHECK ? nch0 : nch0 - 1;
  constexpr int WC = kWalkWin / C;               // chunks per window
  const double a = act ? ca[w] : 0.0, b = act ? cb[w] : 0.0;
  double2* sv = S + w * sstride;
  BihRowState m2 = {0, 0, 0, 0, 0}, m4 = {0, 0, 0, 0, 0};
  int bad = INT_MAX;
  for (int c0 = 0; c0 < cend; c0 += WC) {
    const int i0 = c0 * C;
    __syncthreads();  // the previous window is no longer read
    for (int r = threadIdx.x; r < 2 * kWalkWin; r += blockDim.x) {
      const int k = 2 * i0 + r;
      if (k < N) {
        Recip R;
        R.init(k);
        mats_put(win + r * kWalkWords, bih_mats(k, N, gl, R));
      }
    }
    __syncthreads();
    for (int cc = 0; cc < WC && c0 + cc < cend; ++cc) {
      const int c = c0 + cc;
      // C rows unrolled (rows past the chain, whose window rows may be
      // unset, only feed a recurrence that is not used again)
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const int i = c * C + j;
        const int k = 2 * i + p;
        BihRowState o;
        double l1, l2, t0, sc;
        bih_step_row(bih_row_from(mats_get(win + (k - 2 * i0) * kWalkWords), a, b), m2, m4, o, l1, l2, t0, sc);
        if constexpr (CHECK) bad = first_bad(bad, i < nc && bad_pivot(t0, sc), k);
        m4 = m2;
        m2 = o;
      }
      if (act && c + 1 < nch) {  // the state entering chunk c + 1
        const double v[10] = {m2.rU0, m2.U2, m2.U4, m2.P, m2.R, m4.rU0, m4.U2, m4.U4, m4.P, m4.R};
#pragma unroll
        for (int q = 0; q < 5; ++q)
          sv[ONE ? 2 * (5 * (c + 1) + q) + p : (p * Gt + c + 1) * 5 + q] = make_double2(v[2 * q], v[2 * q + 1]);
      }
    }
  }
  if constexpr (CHECK) {
    if (info != nullptr) walk_info(bad, act, p, w, info);
    if (park && act) park_bad(sv, p, bad);
  }
}

// Lowest bad row over the work group's wavefronts -> info[w].
__device__ __forceinline__ void multi_info(int bad, int v, int W, int lane, int* __restrict__ badw, int32_t* __restrict__ info,
                                           int64_t w) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) bad = min(bad, __shfl_xor(bad, d, 64));
  if (lane == 0) badw[v] = bad;
  __syncthreads();
  if (v == 0 && lane == 0) {
    int b = INT_MAX;
    for (int i = 0; i < W; ++i) b = min(b, badw[i]);
    info[w] = (b == INT_MAX) ? 0 : b + 1;
  }
}

// Work group -> (system, lane's chain parity, lane's chunk in its chain).
// With one parity per work group, the two chains of a system go to blocks 8
// apart (blocks 16q .. 16q + 15 hold systems 8q .. 8q + 7, parity 0 then 1):
// blocks are dealt to the 8 XCDs in turn, so both land on the same XCD and
// share its L2, where the rows of the two parities share cache lines.
template <int W, bool ONE>
struct MultiLane {
  int64_t w;
  int v, lane, h, p, mg;
  __device__ __forceinline__ MultiLane() {
    v = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    lane = threadIdx.x & 63;
    const int64_t b = blockIdx.x;
    w = ONE ? (b >> 4) * 8 + (b & 7) : b;
    h = (lane / kMultiG) & 1;
    p = ONE ? (int)((b >> 3) & 1) : h;
    mg = (ONE ? 2 * v + h : v) * kMultiG + lane % kMultiG;
  }
};
// Blocks of the one-parity grid: 16 per 8 systems (those past nsys exit).
inline int64_t multi_one_blocks(int64_t nsys) { return (nsys + 7) / 8 * 16; }

// States of system w from sts + w sstride.  ONE: info only from the parked
// first bad rows of a factor call (parked_info), else the walk wrote it.
template <int W, bool ONE>
__global__ __launch_bounds__(64 * W) void helm_wave_multi(int N, int64_t nsys, const double* __restrict__ alpha, const double2* __restrict__ f,
                                                          double2* __restrict__ u, const double2* __restrict__ sts,
                                                          int64_t sstride, int gl, int32_t* __restrict__ info,
                                                          int parked_info) {
  constexpr int C = kMultiC, G = kMultiG;
  __shared__ double xch[3 * kCarryMaxW * 2 * kCarryWords];
  __shared__ int badw[kCarryMaxW];
  const MultiLane<W, ONE> L;
  const int64_t w = L.w;
  if (w >= nsys) return;  // the whole work group (padding blocks of the one-parity grid)
  const int n = N - 2;
  const int k0 = 2 * L.mg * C + L.p;
  const double al = alpha[w];
  const double2* frow = f + w * (int64_t)N;
  double2* urow = u + w * (int64_t)N;
  // restart state (every wavefront reads its states before the first
  // barrier of the scans, and stores only after the last)
  const double2* srow = sts + w * sstride;
  HelmPrev pv = {0.0, 0.0};
  if (L.mg > 0 && k0 < n) {
    const double2 s = ONE ? srow[2 * L.mg + L.p] : srow[L.p * W * G + L.mg];
    pv.rd = s.x;
    pv.g = s.y;
  }
  if (ONE && parked_info && info != nullptr && L.p == 0 && threadIdx.x == 0) {
    const int b = min(parked_bad(srow, 0), parked_bad(srow, 1));
    info[w] = (b == INT_MAX) ? 0 : b + 1;
  }
  double2 x[C];
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int k = k0 + 2 * j;
    x[j] = (k < n) ? frow[k] : zero2();
  }
  int bad;
  if constexpr (ONE) {
    const ChainCarry cy{L.v, W, L.p, xch};
    bad = helm_wave_core<C, G, true, ChainCarry>(N, L.lane, w, true, al, pv, x, urow, gl, nullptr, cy);
  } else {
    const WaveCarry cy{L.v, W, xch};
    bad = helm_wave_core<C, G, true, WaveCarry>(N, L.lane, w, true, al, pv, x, urow, gl, nullptr, cy);
  }
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int k = k0 + 2 * j;
    if (k < N) urow[k] = (k < n) ? x[j] : zero2();
  }
  if (!ONE && info != nullptr) multi_info(bad, L.v, W, L.lane, badw, info, w);
}

template <int W, bool ONE>
__global__ __launch_bounds__(64 * W) void bih_wave_multi(int N, int64_t nsys, const double* __restrict__ ca, const double* __restrict__ cb,
                                                         const double2* __restrict__ f, double2* __restrict__ u,
                                                         const double2* __restrict__ sts, int64_t sstride, int gl,
                                                         int32_t* __restrict__ info, int parked_info) {
  constexpr int C = kMultiC, G = kMultiG;
  __shared__ double xch[3 * kCarryMaxW * 2 * kCarryWords];
  __shared__ int badw[kCarryMaxW];
  const MultiLane<W, ONE> L;
  const int64_t w = L.w;
  if (w >= nsys) return;  // the whole work group (padding blocks of the one-parity grid)
  const int n = N - 4;
  const int k0 = 2 * L.mg * C + L.p;
  const double a = ca[w], b = cb[w];
  const double2* frow = f + w * (int64_t)N;
  double2* urow = u + w * (int64_t)N;
  const double2* srow = sts + w * sstride;
  BihRowState m2 = {0, 0, 0, 0, 0}, m4 = {0, 0, 0, 0, 0};
  if (ONE && parked_info && info != nullptr && L.p == 0 && threadIdx.x == 0) {
    const int bq = min(parked_bad(srow, 0), parked_bad(srow, 1));
    info[w] = (bq == INT_MAX) ? 0 : bq + 1;
  }
  if (L.mg > 0 && k0 < n) {
    double2 s[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) s[q] = ONE ? srow[2 * (5 * L.mg + q) + L.p] : srow[(L.p * W * G + L.mg) * 5 + q];
    m2 = BihRowState{s[0].x, s[0].y, s[1].x, s[1].y, s[2].x};
    m4 = BihRowState{s[2].y, s[3].x, s[3].y, s[4].x, s[4].y};
  }
  double2 x[C];
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int k = k0 + 2 * j;
    x[j] = (k < n) ? frow[k] : zero2();
  }
  auto fetch = [&](int j) {
    const int k = k0 + 2 * j;
    return (k < n) ? frow[k] : zero2();
  };
  int bad;
  if constexpr (ONE) {  // the walk has checked every pivot and writes info
    const ChainCarry cy{L.v, W, L.p, xch};
    bad = bih_wave_core<C, G, true, false>(N, L.lane, w, true, a, b, m2, m4, x, fetch, urow, gl, nullptr, nullptr, NoHook(),
                                           std::true_type{}, INT_MAX, cy);
  } else {
    const WaveCarry cy{L.v, W, xch};
    bad = bih_wave_core<C, G, true, false>(N, L.lane, w, true, a, b, m2, m4, x, fetch, urow, gl, nullptr, nullptr, NoHook(),
                                           std::false_type{}, INT_MAX, cy);
  }
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int k = k0 + 2 * j;
    if (k < N) urow[k] = (k < n) ? x[j] : zero2();
  }
  if (!ONE && info != nullptr) multi_info(bad, L.v, W, L.lane, badw, info, w);
}

// =========================================================================
// host side
// =========================================================================

// Chunk length C and lanes per chain G: the first candidate whose 2G lanes
// cover every slot k < N (G*C >= nc = ceil(N/2)) and whose restart states fit
// in one output row (2G chunks x 2 or 10 doubles <= 2N doubles); {0,0} if none.
__host__ __device__ WaveCfg pick_cfg(int nc, int family, int N, int prefC) {
  const WaveCfg helm[] = {{4, 8}, {8, 8}, {8, 16}, {16, 16}, {8, 32}, {16, 32}};
  const WaveCfg bih[] = {{8, 4}, {16, 4}, {8, 8}, {8, 16}, {16, 8}, {16, 16}, {8, 32}, {16, 32}};
  const WaveCfg* list = family == 0 ? helm : bih;
  const int cnt = family == 0 ? 6 : 8;
  const int per = family == 0 ? 2 : 10;
  for (int pass = (prefC > 0 ? 0 : 1); pass < 2; ++pass) {
    for (int i = 0; i < cnt; ++i) {
      const WaveCfg c = list[i];
      if (pass == 0 && c.C != prefC) continue;
      if (c.G * c.C >= nc && per * 2 * c.G <= 2 * N) return c;
    }
  }
  return WaveCfg{0, 0};
}

// opts.chunk: 0 (automatic) or a chunk length some configuration of (family,
// N) is built with
bool wave_chunk_ok(int family, int N, int chunk) {
  if (chunk == 0) return true;
  const WaveCfg c = pick_cfg((N + 1) / 2, family, N, chunk);
  return c.C == chunk;
}

bool wave_supported(int family, int N) {
  const int n = family == 0 ? N - 2 : N - 4;
  if (n < 1) return false;
  const WaveCfg c = pick_cfg((N + 1) / 2, family, N, 0);
  return c.C != 0;
}

// Wavefronts per work group of the large-N solves (0: not served there): N
// past the one-wavefront configurations; two parity chains per work group
// while they fit in kCarryMaxW wavefronts (2048 chain elements), else one
// chain per work group (4096 elements), *one set.
int multi_waves(int family, int N, bool* one) {
  if (one) *one = false;
  if (wave_supported(family, N)) return 0;
  const int per = kMultiC * kMultiG;  // chain elements per G-lane group
  const int nc = (N + 1) / 2;         // the longer chain's bound
  const int W2 = (nc + per - 1) / per;
  if (W2 >= 2 && W2 <= kCarryMaxW) return W2;
  const int W1 = (nc + 2 * per - 1) / (2 * per);
  if (W1 < 2 || W1 > kCarryMaxW) return 0;
  if (one) *one = true;
  return W1;
}

hipError_t launch_multi(const WaveArgs& a) {
  bool one = false;
  const int W = multi_waves(a.family, a.N, &one);
  if (W == 0 || a.mixed || a.adjoint || a.rhs) return hipErrorInvalidValue;
  if (a.nsys <= 0) return hipSuccess;
  // one work group per system (per chain with one parity per work group)
  if ((one ? multi_one_blocks(a.nsys) : a.nsys) > (int64_t)INT_MAX) return hipErrorInvalidValue;
  hipStream_t st = (hipStream_t)a.stream;
  const int Gt = W * kMultiG;
  // restart states in the output row, or in the factor buffer (fac_mode 1:
  // the walk alone, 2: the solve alone)
  double2* S = a.fac_mode ? (double2*)a.fac : (double2*)a.u;
  const int64_t ss = a.fac_mode ? wave_state_slot(a.family, a.N, 0) : (int64_t)a.N;
  if (a.fac_mode != 2) {
    const unsigned walk = (unsigned)((2 * a.nsys + 255) / 256);
    int32_t* winfo = (one && a.fac_mode == 0) ? a.info : nullptr;
    const int park = one && a.fac_mode == 1;
    if (one && a.fac_mode == 0 && a.info == nullptr) {  // the checks only serve info
      if (a.family == 0)
        hipLaunchKernelGGL((helm_walk_multi<true, false>), dim3(walk), dim3(256), 0, st, a.N, a.nsys, Gt, a.c0, S, ss, a.gl,
                           nullptr, 0);
      else
        hipLaunchKernelGGL((bih_walk_multi<true, false>), dim3(walk), dim3(256), 0, st, a.N, a.nsys, Gt, a.c0, a.c1, S, ss,
                           a.gl, nullptr, 0);
    } else if (one) {
      if (a.family == 0)
        hipLaunchKernelGGL(helm_walk_multi<true>, dim3(walk), dim3(256), 0, st, a.N, a.nsys, Gt, a.c0, S, ss, a.gl, winfo, park);
      else
        hipLaunchKernelGGL(bih_walk_multi<true>, dim3(walk), dim3(256), 0, st, a.N, a.nsys, Gt, a.c0, a.c1, S, ss, a.gl, winfo,
                           park);
    } else {
      if (a.family == 0)
        hipLaunchKernelGGL(helm_walk_multi<false>, dim3(walk), dim3(256), 0, st, a.N, a.nsys, Gt, a.c0, S, ss, a.gl, nullptr, 0);
      else
        hipLaunchKernelGGL(bih_walk_multi<false>, dim3(walk), dim3(256), 0, st, a.N, a.nsys, Gt, a.c0, a.c1, S, ss, a.gl, nullptr,
                           0);
    }
  }
  if (a.fac_mode == 1) return hipGetLastError();
  double2* u = (double2*)a.u;
  const double2* f = (const double2*)a.f;
  const int parked = one && a.fac_mode == 2;
  const dim3 grid((unsigned)(one ? multi_one_blocks(a.nsys) : a.nsys)), block(64 * W);
#define SHEN_MULTI(WW, ONE)                                                                                          \
  if (W == WW && one == ONE) {                                                                                       \
    if (a.family == 0)                                                                                               \
      hipLaunchKernelGGL((helm_wave_multi<WW, ONE>), grid, block, 0, st, a.N, a.nsys, a.c0, f, u, S, ss, a.gl, a.info,     \
                         parked);                                                                                    \
    else                                                                                                             \
      hipLaunchKernelGGL((bih_wave_multi<WW, ONE>), grid, block, 0, st, a.N, a.nsys, a.c0, a.c1, f, u, S, ss, a.gl, a.info, \
                         parked);                                                                                    \
  }
  SHEN_MULTI(2, false)
  SHEN_MULTI(3, false)
  SHEN_MULTI(4, false)
  SHEN_MULTI(3, true)
  SHEN_MULTI(4, true)
#undef SHEN_MULTI
  return hipGetLastError();
}

// Systems per boundary/solve launch pair.  Smaller slices keep the restart
// states in the last-level cache, but starve the sequential boundary kernel
// of waves; measured slower at the channel-scale sizes, so off.
static constexpr int64_t kWaveSlice = (int64_t)1 << 40;  // no slicing: boundary kernels need the whole grid for occupancy

// Allows a kernel dynamic LDS beyond the default 64 KiB.
static bool set_dynamic_lds(const void* kernel, size_t bytes) {
  return hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess;
}

// Grid of a persistent kernel: every resident wavefront slot of the device,
// capped by the number of work groups.
static int64_t persistent_blocks(const void* kernel, int64_t groups, int threads = 64, size_t lds = 0) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) != hipSuccess || per_cu < 1) per_cu = 1;
  const int64_t slots = (int64_t)cus * per_cu;
  return groups < slots ? (groups > 0 ? groups : 1) : slots;
}

template <int C, int G>
static hipError_t launch_helm_t(const WaveArgs& a) {
  constexpr int SPW = 64 / (2 * G);
  hipStream_t st = (hipStream_t)a.stream;
  for (int64_t s0 = 0; s0 < a.nsys; s0 += kWaveSlice) {
    const int64_t ns = (a.nsys - s0 < kWaveSlice) ? a.nsys - s0 : kWaveSlice;
    const double* c0 = a.c0 + s0;
    const double2* f = (const double2*)a.f + s0 * a.N;
    double2* u = (double2*)a.u + s0 * a.N;
    int32_t* info = a.info ? a.info + s0 : nullptr;
    const int64_t groups = (ns + SPW - 1) / SPW;
    if (a.adjoint) {
      // restart states: parked in lambda, or the forward solve's (factor-once mode)
      constexpr int64_t kSlotA = 2 * G;
      double2* sts = a.fac_mode ? (double2*)a.fac + s0 * kSlotA : u;
      const int64_t sstride = a.fac_mode ? kSlotA : (int64_t)a.N;
      if (a.fac_mode == 0)
        hipLaunchKernelGGL((helm_boundary_t<C, G>), dim3((unsigned)((2 * ns + 255) / 256)), dim3(256), 0, st, a.N, ns, c0, u,
                           (int64_t)a.N, a.gl);
      hipLaunchKernelGGL((helm_adjoint_wave<C, G>), dim3((unsigned)groups), dim3(64), 0, st, a.N, ns, c0,
                         a.ufwd ? (const double2*)a.ufwd + s0 * a.N : nullptr, f, u, sts, sstride, a.g0 ? a.g0 + s0 : nullptr,
                         a.gl, info);
      continue;
    }
    if (a.mixed) {
      hipLaunchKernelGGL(helm_boundary32, dim3((unsigned)((2 * ns + 255) / 256)), dim3(256), 0, st, a.N, ns, C, G, c0, u, a.gl);
      hipLaunchKernelGGL((helm_mixed_wave<C, G>), dim3((unsigned)groups), dim3(64), 0, st, a.N, ns, c0, f, u, a.gl, info,
                         a.iters ? a.iters + s0 : nullptr, a.it_max, a.tol);
      continue;
    }
    // restart states: parked in u (one call), or in the caller's slots (factor-once mode)
    constexpr int64_t kSlot = 2 * G;  // double2 per system
    double2* sts = a.fac_mode ? (double2*)a.fac + s0 * kSlot : u;
    const int64_t sstride = a.fac_mode ? kSlot : (int64_t)a.N;
    if (a.fac_mode != 2)
      hipLaunchKernelGGL((helm_boundary_t<C, G>), dim3((unsigned)((2 * ns + 255) / 256)), dim3(256), 0, st, a.N, ns, c0, sts,
                         sstride, a.gl);
    if (a.fac_mode == 1) continue;
    if constexpr (C >= 8 && C % 4 == 0 && G >= 16) {
      const int64_t blocks = persistent_blocks((const void*)helm_wave_pipe<C, G>, groups);
      hipLaunchKernelGGL((helm_wave_pipe<C, G>), dim3((unsigned)blocks), dim3(64), 0, st, a.N, ns, c0, f, u, sts, sstride, a.gl,
                         info);
    } else {
      hipLaunchKernelGGL((helm_wave_solve<C, G>), dim3((unsigned)groups), dim3(64), 0, st, a.N, ns, c0, f, u, sts, sstride, a.gl,
                         info);
    }
  }
  return hipGetLastError();
}

template <int C, int G>
static hipError_t launch_bih_t(const WaveArgs& a) {
  constexpr int SPW = 64 / (2 * G);
  hipStream_t st = (hipStream_t)a.stream;
  for (int64_t s0 = 0; s0 < a.nsys; s0 += kWaveSlice) {
    const int64_t ns = (a.nsys - s0 < kWaveSlice) ? a.nsys - s0 : kWaveSlice;
    const double* c0 = a.c0 + s0;
    const double* c1 = a.c1 + s0;
    const double2* f = (const double2*)a.f + s0 * a.N;
    double2* u = (double2*)a.u + s0 * a.N;
    int32_t* info = a.info ? a.info + s0 : nullptr;
    const size_t lds = (size_t)bih_tab_pairs(2 * G * C) * 2 * G * C * sizeof(double2);
    if (a.adjoint) {
      // + the multipliers (and the reciprocal pivots)
      const size_t ldsa = lds + (size_t)C * 256 * (sizeof(double2) + (AdjR0Lds<G>::value ? sizeof(double) : 0));
      static const bool attra = set_dynamic_lds((const void*)bih_adjoint_tab<C, G>, ldsa) &&
                                set_dynamic_lds((const void*)bih_boundary_tab<C, G, false>, lds);
      (void)attra;
      // restart states: parked in lambda, or the forward solve's (factor-once mode)
      constexpr int64_t kSlotA = 2 * G * 5;
      double2* sts = a.fac_mode ? (double2*)a.fac + s0 * kSlotA : u;
      const int64_t sstride = a.fac_mode ? kSlotA : (int64_t)a.N;
      if (a.fac_mode == 0)
        hipLaunchKernelGGL((bih_boundary_tab<C, G, false>), dim3((unsigned)((ns + kBihWalkSystems - 1) / kBihWalkSystems)),
                           dim3(kBihWalkThreads), lds, st, a.N, ns, c0, c1, u, (int64_t)a.N, a.gl);
      hipLaunchKernelGGL((bih_adjoint_tab<C, G>), dim3((unsigned)((ns + 4 * SPW - 1) / (4 * SPW))), dim3(256), ldsa, st, a.N, ns,
                         c0, c1, a.ufwd ? (const double2*)a.ufwd + s0 * a.N : nullptr, f, u, sts, sstride,
                         a.g0 ? a.g0 + s0 : nullptr, a.g1 ? a.g1 + s0 : nullptr, a.gl, info);
      continue;
    }
    if (a.mixed) {
      // the FP32 + refinement kernel and its walk keep the full row table
      const size_t ldsf = (size_t)6 * 2 * G * C * sizeof(double2);
      const size_t ldsm = ldsf + (size_t)4 * 64 * 10 * sizeof(double) + MixedTile<C, G>::bytes;
      static const bool attrm = set_dynamic_lds((const void*)bih_mixed_tab<C, G>, ldsm) &&
                                set_dynamic_lds((const void*)bih_boundary_tab<C, G, true>, ldsf);
      (void)attrm;
      hipLaunchKernelGGL((bih_boundary_tab<C, G, true>), dim3((unsigned)((ns + kBihWalkSystems - 1) / kBihWalkSystems)),
                         dim3(kBihWalkThreads), ldsf, st, a.N, ns, c0, c1, u,
                         (int64_t)a.N, a.gl);
      hipLaunchKernelGGL((bih_mixed_tab<C, G>), dim3((unsigned)((ns + 4 * SPW - 1) / (4 * SPW))), dim3(256), ldsm, st, a.N, ns, c0,
                         c1, f, u, a.gl, info, a.iters ? a.iters + s0 : nullptr, a.it_max, a.tol);
      continue;
    }
    static const bool attr = set_dynamic_lds((const void*)bih_wave_tab<C, G>, lds) &&
                             set_dynamic_lds((const void*)bih_boundary_tab<C, G, false>, lds) &&
                             set_dynamic_lds((const void*)bih_boundary_tab<C, G, false, false>, lds) &&
                             set_dynamic_lds((const void*)bih_boundary_tab<C, G, true>, lds);
    (void)attr;
    // restart states: parked in u (one call), or in the caller's slots (factor-once mode)
    constexpr int64_t kSlot = 2 * G * 5;  // double2 per system
    double2* sts = a.fac_mode ? (double2*)a.fac + s0 * kSlot : u;
    const int64_t sstride = a.fac_mode ? kSlot : (int64_t)a.N;
    const dim3 wgrid((unsigned)((ns + kBihWalkSystems - 1) / kBihWalkSystems));
    // the pivot checks serve info only: a one-call solve without info skips them
    if (a.fac_mode == 0 && info == nullptr)
      hipLaunchKernelGGL((bih_boundary_tab<C, G, false, false>), wgrid, dim3(kBihWalkThreads), lds, st, a.N, ns, c0, c1, sts,
                         sstride, a.gl);
    else if (a.fac_mode != 2)
      hipLaunchKernelGGL((bih_boundary_tab<C, G, false>), wgrid, dim3(kBihWalkThreads), lds, st, a.N, ns, c0, c1, sts, sstride,
                         a.gl);
    if (a.fac_mode == 1) continue;
    // gfx950: 160 KiB of LDS per work group
    constexpr int kWpb = PtabWaves<C, G>::value;
    constexpr size_t kPtabLds =
        (size_t)bih_tab_pairs(2 * G * C) * 2 * G * C * sizeof(double2) + (size_t)kWpb * (C + 6) * 64 * sizeof(double2);
    if constexpr (C >= 8 && C % 4 == 0 && G >= 16 && kPtabLds <= 160 * 1024) {
      const size_t lds2 = kPtabLds;
      static const bool attr2 = set_dynamic_lds((const void*)bih_wave_ptab<C, G>, lds2);
      (void)attr2;
      const int64_t groups = (ns + SPW - 1) / SPW;
      const int64_t blocks =
          persistent_blocks((const void*)bih_wave_ptab<C, G>, (groups + kWpb - 1) / kWpb, 64 * kWpb, lds2);
      hipLaunchKernelGGL((bih_wave_ptab<C, G>), dim3((unsigned)blocks), dim3(64 * kWpb), lds2, st, a.N, ns, c0, c1, f, u, sts,
                         sstride, a.gl, info);
    } else {
      hipLaunchKernelGGL((bih_wave_tab<C, G>), dim3((unsigned)((ns + 4 * SPW - 1) / (4 * SPW))), dim3(256), lds, st, a.N, ns, c0,
                         c1, f, u, sts, sstride, a.gl, info);
    }
  }
  return hipGetLastError();
}

template <int C, int G>
static hipError_t launch_matvec_t(const WaveArgs& a) {
  constexpr int SPW = 64 / (2 * G);
  if constexpr (!(C >= 8 && C % 4 == 0 && G >= 16)) {
    return hipErrorInvalidValue;
  } else {
    hipStream_t st = (hipStream_t)a.stream;
    const int64_t groups = (a.nsys + SPW - 1) / SPW;
    const double2* uin = (const double2*)a.f;
    double2* hu = (double2*)a.u;
    const double2* sh = (const double2*)a.sh;
    if (a.family == 0) {
      if (a.rhs) {
        const int64_t blocks = persistent_blocks((const void*)helm_matvec_pipe<C, G, true>, groups);
        hipLaunchKernelGGL((helm_matvec_pipe<C, G, true>), dim3((unsigned)blocks), dim3(64), 0, st, a.N, a.nsys, a.c0, uin, hu,
                           a.gl, a.inv, a.sigma, sh);
      } else {
        const int64_t blocks = persistent_blocks((const void*)helm_matvec_pipe<C, G>, groups);
        hipLaunchKernelGGL((helm_matvec_pipe<C, G>), dim3((unsigned)blocks), dim3(64), 0, st, a.N, a.nsys, a.c0, uin, hu, a.gl,
                           0.0, 0.0, nullptr);
      }
    } else {
      constexpr size_t lds = (size_t)bih_tab_pairs(2 * G * C) * 2 * G * C * sizeof(double2) + (size_t)4 * (C + 1) * 64 * sizeof(double2);
      if constexpr (lds > 160 * 1024) {
        return hipErrorInvalidValue;
      } else if (a.rhs) {
        static const bool attr = set_dynamic_lds((const void*)bih_matvec_ptab<C, G, true>, lds);
        (void)attr;
        const int64_t blocks = persistent_blocks((const void*)bih_matvec_ptab<C, G, true>, (groups + 3) / 4, 256, lds);
        hipLaunchKernelGGL((bih_matvec_ptab<C, G, true>), dim3((unsigned)blocks), dim3(256), lds, st, a.N, a.nsys, a.c0, a.c0,
                           uin, hu, a.gl, a.inv, a.sigma, sh);
      } else {
        static const bool attr = set_dynamic_lds((const void*)bih_matvec_ptab<C, G>, lds);
        (void)attr;
        const int64_t blocks = persistent_blocks((const void*)bih_matvec_ptab<C, G>, (groups + 3) / 4, 256, lds);
        hipLaunchKernelGGL((bih_matvec_ptab<C, G>), dim3((unsigned)blocks), dim3(256), lds, st, a.N, a.nsys, a.c0, a.c1, uin,
                           hu, a.gl, 0.0, 0.0, nullptr);
      }
    }
    return hipGetLastError();
  }
}

// Configuration of the wave-layout matvec for (family, N): that of the solve.
static WaveCfg matvec_cfg(int family, int N) {
  const int nc = (N + 1) / 2;
  return pick_cfg(nc, family, N, 0);
}

// True when (family, N) has a wave-layout matvec (the tile layout needs
// G >= 16 lanes per chain and C >= 8 rows per chunk, and the biharmonic row
// table plus four tiles must fit the LDS); false otherwise (the caller then
// uses the chain kernels).
bool matvec_wave_supported(int family, int N) {
  const WaveCfg c = matvec_cfg(family, N);
  if (!(c.C >= 8 && c.C % 4 == 0 && c.G >= 16)) return false;
  const size_t lds = (size_t)bih_tab_pairs(2 * c.G * c.C) * 2 * c.G * c.C * sizeof(double2) + (size_t)4 * (c.C + 1) * 64 * sizeof(double2);
  return family == 0 || lds <= 160 * 1024;
}

hipError_t launch_matvec_wave(const WaveArgs& a) {
  if (a.nsys <= 0) return hipSuccess;
  const WaveCfg c = matvec_cfg(a.family, a.N);
#define SHEN_MV(CC, GG) \
  if (c.C == CC && c.G == GG) return launch_matvec_t<CC, GG>(a);
  SHEN_MV(8, 16)
  SHEN_MV(16, 16)
  SHEN_MV(8, 32)
  SHEN_MV(16, 32)
#undef SHEN_MV
  return hipErrorInvalidValue;
}

// Mass-matrix solves: the configuration by N (the tile layout needs G >= 16
// lanes per chain and C >= 8 rows per chunk); C = 0 beyond N = 1024.
static WaveCfg mass_cfg(int family, int N) {
  (void)family;  // both bases take the same configurations
  const int nc = (N + 1) / 2;
  if (nc <= 128) return WaveCfg{8, 16};
  if (nc <= 256) return WaveCfg{16, 16};
  if (nc <= 512) return WaveCfg{16, 32};
  return WaveCfg{0, 0};
}
bool mass_wave_supported(int N) { return mass_cfg(0, N).C != 0 && mass_cfg(1, N).C != 0; }

template <int C, int G, int FAM, int OP>
static hipError_t launch_mass_t(const WaveArgs& a) {
  using L = MassLds<C, G, FAM, OP>;
  static_assert(L::bytes <= 160 * 1024, "mass-solve LDS beyond the work-group limit");
  constexpr int SPW = 64 / (2 * G);
  static const bool attr = set_dynamic_lds((const void*)mass_wave_pipe<C, G, FAM, OP>, L::bytes);
  (void)attr;
  const int64_t groups = (a.nsys + SPW - 1) / SPW;
  const int64_t blocks = persistent_blocks((const void*)mass_wave_pipe<C, G, FAM, OP>, (groups + L::WPB - 1) / L::WPB,
                                           64 * L::WPB, L::bytes);
  hipLaunchKernelGGL((mass_wave_pipe<C, G, FAM, OP>), dim3((unsigned)blocks), dim3(64 * L::WPB), L::bytes, (hipStream_t)a.stream,
                     a.N, a.nsys, (const double2*)a.f, (double2*)a.u, a.gl);
  return hipGetLastError();
}

hipError_t launch_mass_wave(const WaveArgs& a) {
  if (a.nsys <= 0) return hipSuccess;
  const WaveCfg c = mass_cfg(a.family, a.N);
#define SHEN_MASS(CC, GG) \
  if (c.C == CC && c.G == GG)                                                                              \
    return a.family == 1 ? launch_mass_t<CC, GG, 1, 0>(a) : a.deriv ? launch_mass_t<CC, GG, 0, 1>(a) : launch_mass_t<CC, GG, 0, 0>(a);
  SHEN_MASS(8, 16)
  SHEN_MASS(16, 16)
  SHEN_MASS(8, 32)
  SHEN_MASS(16, 32)
#undef SHEN_MASS
  return hipErrorInvalidValue;
}

// double2 per system of the factor-once state slots (0: no wave kernel for N)
int64_t wave_state_slot(int family, int N, int chunk) {
  const WaveCfg c = pick_cfg((N + 1) / 2, family, N, chunk);
  if (c.C != 0) return (int64_t)2 * c.G * (family == 0 ? 1 : 5);
  // large N: W G chunks per chain and wavefront group; with one parity per
  // work group the 2 W G chunks of a chain are interleaved by parity
  bool one = false;
  const int W = chunk == 0 ? multi_waves(family, N, &one) : 0;
  if (W == 0) return 0;
  return (int64_t)(one ? 4 : 2) * W * kMultiG * (family == 0 ? 1 : 5);
}

hipError_t launch_wave(const WaveArgs& a) {
  const int n = a.family == 0 ? a.N - 2 : a.N - 4;
  (void)n;
  const WaveCfg c = pick_cfg((a.N + 1) / 2, a.family, a.N, a.chunk);
  if (a.nsys <= 0) return hipSuccess;
#define SHEN_DISPATCH(CC, GG)                                                         \
  if (c.C == CC && c.G == GG) return a.family == 0 ? launch_helm_t<CC, GG>(a) : launch_bih_t<CC, GG>(a);
  SHEN_DISPATCH(4, 8)
  SHEN_DISPATCH(8, 4)
  SHEN_DISPATCH(16, 4)
  SHEN_DISPATCH(8, 8)
  SHEN_DISPATCH(8, 16)
  SHEN_DISPATCH(16, 8)
  SHEN_DISPATCH(16, 16)
  SHEN_DISPATCH(8, 32)
  SHEN_DISPATCH(16, 32)
#undef SHEN_DISPATCH
  return hipErrorInvalidValue;
}


// =========================================================================
// Batched form: many grids of uneven N and both families.  The host groups
// the grids by class (family, N, wave configuration) and enqueues, per class,
// the kernels of the single-grid path over all of the class's grids at once:
// the boundary walk, then the wave solve (the persistent LDS-streamed
// helm_wave_pipe / table-driven bih_wave_ptab bodies where the configuration
// has them, the per-group kernels otherwise).  A launch takes up to kMaxSeg
// grids in a segment table passed by value; their groups (and walk blocks)
// are numbered grid after grid.  The persistent solves pull work items of
// `gpi` consecutive groups of one grid from their own counter in the caller's
// work buffer (cleared by the first kernel of the call), so every launch is
// graph-capturable and every wavefront reaches the exit once the queue is
// empty.
// =========================================================================
// Arrays of one grid of a batched launch (restart states parked in u).
struct GridRef {
  int64_t nsys;
  const double* c0;
  const double* c1;
  const double2* f;
  double2* u;
  int32_t* info;
};

static constexpr int kMaxSeg = 16;
// The grids of one batched launch: items (of gpi groups) and walk blocks
// numbered one grid after the other; ibeg[nseg] and bbeg[nseg] are the totals.
struct SegSrc {
  int nseg;
  int gpi;  // groups per work item of the persistent solves
  int64_t ibeg[kMaxSeg + 1];
  int64_t bbeg[kMaxSeg + 1];
  GridRef r[kMaxSeg];
};

// Segment holding virtual index v of a prefix table (uniform: scalar loads
// of the kernel argument).
__device__ __forceinline__ int seg_of(const int64_t* beg, int nseg, int64_t v) {
  int s = 0;
  for (int i = 1; i < nseg; ++i) s = (v >= beg[i]) ? i : s;
  return s;
}

__global__ void batched_clear(unsigned long long* __restrict__ counter, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) counter[i] = 0ULL;
}

// Next work item for this wavefront (one atomic per item, lane 0).
__device__ __forceinline__ int64_t pull_item(unsigned long long* __restrict__ counter) {
  unsigned long long t = 0;
  if ((threadIdx.x & 63) == 0) t = atomicAdd(counter, 1ULL);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)t), hi = __builtin_amdgcn_readfirstlane((unsigned)(t >> 32));
  return (int64_t)(((unsigned long long)hi << 32) | lo);
}

// ---------------------------------------------------------------- walks
template <int C, int G>
__global__ __launch_bounds__(256) void batched_helm_walk(int N, SegSrc src, int gl) {
  const int64_t vb = blockIdx.x;
  const int s = seg_of(src.bbeg, src.nseg, vb);
  const GridRef& r = src.r[s];
  helm_walk_block<C, G>(N, r.nsys, r.c0, r.u, (int64_t)N, gl, vb - src.bbeg[s]);
}

template <int C, int G>
__global__ __launch_bounds__(kBihWalkThreads) void batched_bih_walk(int N, SegSrc src, int gl) {
  extern __shared__ double tab[];
  bih_tab_fill(tab, 2 * G * C, C, N, gl, threadIdx.x, kBihWalkThreads);
  __syncthreads();
  const int64_t vb = blockIdx.x;
  const int s = seg_of(src.bbeg, src.nseg, vb);
  const GridRef& r = src.r[s];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t w = (vb - src.bbeg[s]) * kBihWalkSystems + (wv >> 1) * 64 + lane;
  if (w >= r.nsys) return;
  bih_walk_tab<C, G, false>(N, wv & 1, r.c0[w], r.c1[w], r.u + w * (int64_t)N, gl, tab);
}

// ------------------------------------------------ per-group wave solves
// (configurations without the tile layout: one group per wavefront)
template <int C, int G>
__global__ __launch_bounds__(64) void batched_helm_solve(int N, SegSrc src, int gl) {
  constexpr int SPW = 64 / (2 * G);
  const int64_t vg = blockIdx.x;  // items of one group (gpi = 1)
  const int s = seg_of(src.ibeg, src.nseg, vg);
  const GridRef& r = src.r[s];
  helm_wave_body<C, G>(N, r.nsys, (vg - src.ibeg[s]) * SPW, r.c0, r.f, r.u, r.u, (int64_t)N, gl, r.info);
}

template <int C, int G>
__global__ __launch_bounds__(256) void batched_bih_solve(int N, SegSrc src, int gl) {
  extern __shared__ double tab[];
  constexpr int SPW = 64 / (2 * G);
  bih_tab_fill(tab, 2 * G * C, C, N, gl, threadIdx.x, 256);
  __syncthreads();
  const int64_t vg = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (vg >= src.ibeg[src.nseg]) return;
  const int s = seg_of(src.ibeg, src.nseg, vg);
  const GridRef& r = src.r[s];
  bih_wave_body<C, G, true>(N, r.nsys, (vg - src.ibeg[s]) * SPW, r.c0, r.c1, r.f, r.u, r.u, (int64_t)N, gl, r.info, tab);
}

// --------------------------------------- persistent LDS-streamed solves
// The bodies of helm_wave_pipe / bih_wave_ptab over a dynamic queue of work
// items; the next group (of this item, or the first of the next one) streams
// into the tile while the current one is solved.
struct GroupCursor {
  int64_t item, g, gend;  // current item, group within its grid, end of item
  int s;                  // segment
};
__device__ __forceinline__ bool cursor_at(const SegSrc& src, int spw, int64_t item, GroupCursor& c) {
  if (item >= src.ibeg[src.nseg]) return false;
  c.item = item;
  c.s = seg_of(src.ibeg, src.nseg, item);
  const int64_t groups = (src.r[c.s].nsys + spw - 1) / spw;
  c.g = (item - src.ibeg[c.s]) * src.gpi;
  c.gend = c.g + src.gpi < groups ? c.g + src.gpi : groups;
  return true;
}
__device__ __forceinline__ bool cursor_next(const SegSrc& src, int spw, unsigned long long* counter, GroupCursor& c) {
  if (c.g + 1 < c.gend) {
    ++c.g;
    return true;
  }
  return cursor_at(src, spw, pull_item(counter), c);
}

template <int C, int G>
__global__ __launch_bounds__(64, 2) void batched_helm_pipe(int N, SegSrc src, unsigned long long* __restrict__ counter, int gl) {
  using TL = Tile<C, G>;
  constexpr int SPW = TL::SPW;
  __shared__ double2 tile[(C + 1) * 64];
  const int n = N - 2;
  GroupCursor cur;
  if (!cursor_at(src, SPW, pull_item(counter), cur)) return;
  auto coef = [&](const GroupCursor& c, int l) {
    const GridRef& r = src.r[c.s];
    const int64_t w = c.g * SPW + l / (2 * G);
    return r.c0[w < r.nsys ? w : r.nsys - 1];
  };
  double2 x[C], st[1];
  double al;
  {
    const int lane = threadIdx.x & 63;
    const GridRef& r = src.r[cur.s];
    prefetch_tile<C, G, 1>(tile, lane, cur.g, N, r.nsys, r.f, r.u, (int64_t)N);
    al = coef(cur, lane);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    read_tile<C, G, 1>(tile, lane, x, st);
  }
  for (;;) {
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));
    lane &= 63;  // opaque, but known to be a lane index
    GroupCursor nxt = cur;
    const bool more = cursor_next(src, SPW, counter, nxt);
    const GridRef& r = src.r[cur.s];
    const int sl = lane / (2 * G), p = (lane / G) & 1, m = lane % G;
    const int k0 = 2 * m * C + p;
    const int64_t w = cur.g * SPW + sl;
    const bool wok = w < r.nsys;
#pragma unroll
    for (int j = 0; j < C; ++j) x[j] = (wok && k0 + 2 * j < n) ? x[j] : zero2();
    HelmPrev pv = {0.0, 0.0};
    if (wok && m > 0 && k0 < n) {
      pv.rd = st[0].x;
      pv.g = st[0].y;
    }
    helm_wave_core<C, G, true>(N, lane, w, wok, wok ? al : 0.0, pv, x, r.u, gl, r.info);
    stage_tile<C, G>(tile, lane, x);
    store_tile<C, G>(tile, lane, cur.g, N, n, r.nsys, r.u);
    if (!more) break;
    cur = nxt;
    const GridRef& rn = src.r[cur.s];
    prefetch_tile<C, G, 1>(tile, lane, cur.g, N, rn.nsys, rn.f, rn.u, (int64_t)N);
    al = coef(cur, lane);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    read_tile<C, G, 1>(tile, lane, x, st);
  }
}

template <int C, int G>
__global__ __launch_bounds__((64 * PtabWaves<C, G>::value)) void batched_bih_ptab(int N, SegSrc src,
                                                                              unsigned long long* __restrict__ counter, int gl) {
  using TL = Tile<C, G>;
  constexpr int SPW = TL::SPW;
  constexpr int RT = 2 * G * C;
  extern __shared__ double smem[];
  double* tab = smem;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  double2* tile = reinterpret_cast<double2*>(smem + 2 * bih_tab_pairs(RT) * RT) + wv * ((C + 6) * 64);
  double2* coef = tile + (C + 5) * 64;
  constexpr int WPB = PtabWaves<C, G>::value;
  bih_tab_fill(tab, RT, C, N, gl, threadIdx.x, 64 * WPB);
  __syncthreads();
  const int n = N - 4;
  GroupCursor cur;
  if (!cursor_at(src, SPW, pull_item(counter), cur)) return;
  auto sysc = [&](const GroupCursor& c, int l) {
    const int64_t w = c.g * SPW + l / (2 * G);
    const int64_t ns = src.r[c.s].nsys;
    return w < ns ? w : ns - 1;
  };
  {
    const int lane = threadIdx.x & 63;
    const GridRef& r = src.r[cur.s];
    prefetch_tile<C, G, 5>(tile, lane, cur.g, N, r.nsys, r.f, r.u, (int64_t)N);
    prefetch_coef2(coef, lane, sysc(cur, lane), r.c0, r.c1);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  }
  for (;;) {
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));
    lane &= 63;  // opaque, but known to be a lane index
    GroupCursor nxt = cur;
    const bool more = cursor_next(src, SPW, counter, nxt);
    const GridRef& r = src.r[cur.s];
    const int sl = lane / (2 * G), p = (lane / G) & 1, m = lane % G;
    const int k0 = 2 * m * C + p;
    const int64_t w = cur.g * SPW + sl;
    const bool wok = w < r.nsys;
    double2 x[C], st[5];
    read_states_asm<C, 5>(tile, lane, st);
    double ca_, cb_;
    read_coef2(coef, lane, ca_, cb_);
    BihRowState m2 = {0, 0, 0, 0, 0}, m4 = {0, 0, 0, 0, 0};
    if (wok && m > 0 && k0 < n) {
      m2 = BihRowState{st[0].x, st[0].y, st[1].x, st[1].y, st[2].x};
      m4 = BihRowState{st[2].y, st[3].x, st[3].y, st[4].x, st[4].y};
    }
    TileFetch4<C, G> fetch;
    fetch.base = (uint32_t)(uintptr_t)SHEN_LDS(tile);
    fetch.sl = sl;
    fetch.k0 = k0;
    fetch.n = n;
    fetch.wok = wok;
    auto prefetch_next = [&]() {
      if (more) {
        const GridRef& rn = src.r[nxt.s];
        prefetch_tile<C, G, 5>(tile, lane, nxt.g, N, rn.nsys, rn.f, rn.u, (int64_t)N);
        prefetch_coef2(coef, lane, sysc(nxt, lane), rn.c0, rn.c1);
      }
    };
    double2* urow = r.u + (wok ? w : 0) * (int64_t)N;
    bih_wave_core<C, G, true, true>(N, lane, w, wok, wok ? ca_ : 0.0, wok ? cb_ : 0.0, m2, m4, x, fetch, urow, gl, r.info, tab,
                                    prefetch_next, std::true_type{}, walk_bad_of(st[0].x, wok && m == 0));
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    if (wok) {
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const int k = k0 + 2 * j;
        if (k < N) urow[k] = x[j];
      }
    }
    if (!more) break;
    cur = nxt;
  }
}

// ------------------------------------------------------------- launcher
namespace {
// Systems per block of the walk kernels, and whether a configuration has the
// LDS-streamed persistent solve.
constexpr int kHelmWalkSystems = 128;
template <int C, int G>
constexpr bool has_tile_layout() {
  return C >= 8 && C % 4 == 0 && G >= 16;
}
template <int C, int G>
constexpr size_t ptab_lds() {
  return (size_t)bih_tab_pairs(2 * G * C) * 2 * G * C * sizeof(double2) + (size_t)PtabWaves<C, G>::value * (C + 6) * 64 * sizeof(double2);
}

// Launches one class (family FAM, configuration C, G, one N) over up to
// kMaxSeg grids; `counter` is this launch's queue counter.
template <int C, int G, int FAM>
hipError_t launch_class(int N, SegSrc& src, unsigned long long* counter, int gl, hipStream_t st) {
  constexpr int SPW = 64 / (2 * G);
  const int walk_sys = FAM == SHEN_HELMHOLTZ ? kHelmWalkSystems : kBihWalkSystems;
  int64_t items = 0, blocks = 0;
  for (int i = 0; i < src.nseg; ++i) {
    src.ibeg[i] = items;
    src.bbeg[i] = blocks;
    const int64_t groups = (src.r[i].nsys + SPW - 1) / SPW;
    items += (groups + src.gpi - 1) / src.gpi;
    blocks += (src.r[i].nsys + walk_sys - 1) / walk_sys;
  }
  src.ibeg[src.nseg] = items;
  src.bbeg[src.nseg] = blocks;
  if (items == 0) return hipSuccess;
  if constexpr (FAM == SHEN_HELMHOLTZ) {
    hipLaunchKernelGGL((batched_helm_walk<C, G>), dim3((unsigned)blocks), dim3(256), 0, st, N, src, gl);
    if constexpr (has_tile_layout<C, G>()) {
      const int64_t grid = persistent_blocks((const void*)batched_helm_pipe<C, G>, items);
      hipLaunchKernelGGL((batched_helm_pipe<C, G>), dim3((unsigned)grid), dim3(64), 0, st, N, src, counter, gl);
    } else {
      SegSrc one = src;  // per-group kernel: one group per item
      one.gpi = 1;
      int64_t g = 0;
      for (int i = 0; i < one.nseg; ++i) {
        one.ibeg[i] = g;
        g += (one.r[i].nsys + SPW - 1) / SPW;
      }
      one.ibeg[one.nseg] = g;
      hipLaunchKernelGGL((batched_helm_solve<C, G>), dim3((unsigned)g), dim3(64), 0, st, N, one, gl);
    }
  } else {
    const size_t lds = (size_t)bih_tab_pairs(2 * G * C) * 2 * G * C * sizeof(double2);
    static const bool attr = set_dynamic_lds((const void*)batched_bih_walk<C, G>, lds) &&
                             set_dynamic_lds((const void*)batched_bih_solve<C, G>, lds);
    (void)attr;
    hipLaunchKernelGGL((batched_bih_walk<C, G>), dim3((unsigned)blocks), dim3(kBihWalkThreads), lds, st, N, src, gl);
    if constexpr (has_tile_layout<C, G>() && ptab_lds<C, G>() <= 160 * 1024) {
      constexpr int kWpb = PtabWaves<C, G>::value;
      constexpr size_t plds = ptab_lds<C, G>();
      static const bool attr2 = set_dynamic_lds((const void*)batched_bih_ptab<C, G>, plds);
      (void)attr2;
      const int64_t grid = persistent_blocks((const void*)batched_bih_ptab<C, G>, (items + kWpb - 1) / kWpb, 64 * kWpb, plds);
      hipLaunchKernelGGL((batched_bih_ptab<C, G>), dim3((unsigned)grid), dim3(64 * kWpb), plds, st, N, src, counter, gl);
    } else {
      SegSrc one = src;
      one.gpi = 1;
      int64_t g = 0;
      for (int i = 0; i < one.nseg; ++i) {
        one.ibeg[i] = g;
        g += (one.r[i].nsys + SPW - 1) / SPW;
      }
      one.ibeg[one.nseg] = g;
      hipLaunchKernelGGL((batched_bih_solve<C, G>), dim3((unsigned)((g + 3) / 4)), dim3(256), lds, st, N, one, gl);
    }
  }
  return hipGetLastError();
}

using ClassLaunch = hipError_t (*)(int, SegSrc&, unsigned long long*, int, hipStream_t);
template <int FAM>
ClassLaunch class_launcher(WaveCfg c) {
#define SHEN_CLASS(CC, GG) \
  if (c.C == CC && c.G == GG) return &launch_class<CC, GG, FAM>;
  SHEN_CLASS(4, 8)
  SHEN_CLASS(8, 4)
  SHEN_CLASS(16, 4)
  SHEN_CLASS(8, 8)
  SHEN_CLASS(16, 8)
  SHEN_CLASS(8, 16)
  SHEN_CLASS(16, 16)
  SHEN_CLASS(8, 32)
  SHEN_CLASS(16, 32)
#undef SHEN_CLASS
  return nullptr;
}
}  // namespace

int batched_counters(int ndesc) { return ndesc > 0 ? ndesc : 0; }

// Groups the (validated, planned) host descriptors by class in descriptor
// order and launches every class over its grids, kMaxSeg at a time.
// Side streams of the batched launch, per device: the classes (each a walk
// and a solve, or several such pairs) are dealt to kForkStreams streams forked
// from the caller's stream and joined back to it before the call returns, so
// that the latency-bound walks and the small classes overlap other classes'
// solves.  Created once per device (default priority, non-blocking), with
// one fork and one join event per stream; the enqueue of a forked call holds
// the lock, so calls from several host threads do not mix their events.  The
// fork/join is graph-capturable (the side streams join the capture and are
// joined back before the call returns).
static constexpr int kForkStreams = 4;
static constexpr int kForkDevices = 64;
struct ForkSet {
  bool ok = false;
  hipStream_t s[kForkStreams];
  hipEvent_t fork;
  hipEvent_t join[kForkStreams];
};
static std::mutex g_fork_mu;
static ForkSet g_fork[kForkDevices];

// The current device's set, created on first use; called with g_fork_mu held.
static hipError_t fork_set_locked(ForkSet** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kForkDevices) return hipErrorInvalidDevice;
  ForkSet& f = g_fork[dev];
  if (!f.ok) {
    for (int i = 0; i < kForkStreams; ++i) {
      if ((e = hipStreamCreateWithFlags(&f.s[i], hipStreamNonBlocking)) != hipSuccess) return e;
      if ((e = hipEventCreateWithFlags(&f.join[i], hipEventDisableTiming)) != hipSuccess) return e;
    }
    if ((e = hipEventCreateWithFlags(&f.fork, hipEventDisableTiming)) != hipSuccess) return e;
    f.ok = true;
  }
  *out = &f;
  return hipSuccess;
}

hipError_t batched_fork_prepare() {
  std::lock_guard<std::mutex> lk(g_fork_mu);
  ForkSet* fs = nullptr;
  return fork_set_locked(&fs);
}

hipError_t launch_batched(const shen_problem* desc, int ndesc, void* work, int gl, void* stream, bool fork) {
  hipStream_t st = (hipStream_t)stream;
  unsigned long long* counter = reinterpret_cast<unsigned long long*>(work);
  const int ncounters = batched_counters(ndesc);
  hipLaunchKernelGGL(batched_clear, dim3(1), dim3(256), 0, st, counter, ncounters);
  std::unique_lock<std::mutex> lk(g_fork_mu, std::defer_lock);
  ForkSet* fs = nullptr;
  if (fork) {
    lk.lock();
    hipError_t e = fork_set_locked(&fs);
    if (e != hipSuccess) return e;
    if ((e = hipEventRecord(fs->fork, st)) != hipSuccess) return e;
    for (int k = 0; k < kForkStreams; ++k)
      if ((e = hipStreamWaitEvent(fs->s[k], fs->fork, 0)) != hipSuccess) return e;
  }
  int ncls = 0;
  auto class_stream = [&]() { return fork ? fs->s[ncls++ % kForkStreams] : st; };
  // every side stream joins the caller's stream again, also after an error
  auto finish = [&](hipError_t err) {
    if (fork) {
      for (int k = 0; k < kForkStreams; ++k) {
        const hipError_t e1 = hipEventRecord(fs->join[k], fs->s[k]);
        const hipError_t e2 = hipStreamWaitEvent(st, fs->join[k], 0);
        if (err == hipSuccess) err = e1 != hipSuccess ? e1 : e2;
      }
    }
    return err != hipSuccess ? err : hipGetLastError();
  };
  std::vector<char> done((size_t)ndesc, 0);
  int slot = 0;
  for (int i = 0; i < ndesc; ++i) {
    if (done[i] || desc[i].nsys <= 0) continue;
    const shen_problem& d = desc[i];
    if (multi_waves(d.family, d.N) > 0) {  // large N: its own walk and solve
      WaveArgs a;
      a.family = d.family;
      a.N = d.N;
      a.nsys = d.nsys;
      a.c0 = d.c0;
      a.c1 = d.c1;
      a.f = d.f;
      a.u = d.u;
      a.info = d.info;
      a.gl = gl;
      a.stream = (void*)class_stream();
      const hipError_t err = launch_multi(a);
      if (err != hipSuccess) return finish(err);
      done[i] = 1;
      continue;
    }
    const WaveCfg c = pick_cfg((d.N + 1) / 2, d.family, d.N, d.chunk);
    ClassLaunch fn = d.family == SHEN_HELMHOLTZ ? class_launcher<SHEN_HELMHOLTZ>(c) : class_launcher<SHEN_BIHARMONIC>(c);
    if (fn == nullptr) return finish(hipErrorInvalidValue);
    const hipStream_t sc = class_stream();
    // groups (of 64 / (2G) systems) per work item
    const int spw = 64 / (2 * c.G);
    auto gpi_of = [&](const shen_problem& e) {
      const int g = (e.sys_per_tile + spw - 1) / spw;
      return g > 0 ? g : 1;
    };
    SegSrc src = {};
    src.gpi = gpi_of(d);
    for (int j = i; j < ndesc; ++j) {
      const shen_problem& e = desc[j];
      if (done[j] || e.nsys <= 0 || e.family != d.family || e.N != d.N) continue;
      const WaveCfg ce = pick_cfg((e.N + 1) / 2, e.family, e.N, e.chunk);
      if (ce.C != c.C || ce.G != c.G || gpi_of(e) != src.gpi) continue;
      done[j] = 1;
      src.r[src.nseg++] = GridRef{e.nsys, e.c0, e.c1, reinterpret_cast<const double2*>(e.f), reinterpret_cast<double2*>(e.u),
                                  e.info};
      if (src.nseg == kMaxSeg) {
        if (slot >= ncounters) return finish(hipErrorInvalidValue);
        const hipError_t err = fn(d.N, src, counter + slot++, gl, sc);
        if (err != hipSuccess) return finish(err);
        src.nseg = 0;
      }
    }
    if (src.nseg > 0) {
      if (slot >= ncounters) return finish(hipErrorInvalidValue);
      const hipError_t err = fn(d.N, src, counter + slot++, gl, sc);
      if (err != hipSuccess) return finish(err);
    }
  }
  return finish(hipSuccess);
}

// ------------------------------------------------------------------------
// Work counters of the batched launch in library-owned device memory, for
// callers that cannot allocate (code under hipGraph capture, serving loops,
// harnesses that forbid hipMalloc).  One array per device, held until the
// process ends; every call on a device shares it, so calls that overlap on
// one device race (the launch clears the counters with its first kernel, so
// what an earlier call left there does not matter).  Host code never passes
// the array's name to a kernel: it stands for a host-side shadow there.  The
// device address is looked up once per device, with that device current.
// ------------------------------------------------------------------------
static __device__ __align__(256) unsigned long long scratch[kBatchedStaticWords];

hipError_t batched_static_scratch(void** ptr) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (addr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

}  // namespace shen
