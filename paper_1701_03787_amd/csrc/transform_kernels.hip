// Wall-normal Shen transforms (Sec. 2; the appendix algorithms for forward
// scalar products / transforms and inverse transforms): Chebyshev, Dirichlet
// (T_k - T_{k+2}) and biharmonic (T_k - 2(k+2)/(k+3) T_{k+2} +
// (k+1)/(k+3) T_{k+4}) bases, at the N Chebyshev-Gauss or
// Chebyshev-Gauss-Lobatto points.
//
//   scalar product  S(u)_k = sum_j u(x_j) phi_k(x_j) sigma_j
//   inverse         u(x_j) = sum_k uhat_k phi_k(x_j)
//
// Both reduce to cosine sums: with C_k = sum_j u_j T_k(x_j) sigma_j the
// scalar products are the Shen combinations C_k - C_{k+2} and C_k -
// 2(k+2)/(k+3) C_{k+2} + (k+1)/(k+3) C_{k+4}; the inverse maps the Shen
// coefficients to Chebyshev ones (the transposed combination) and sums
// z_k T_k(x_j).
//
// Two kernels, one persistent work group of 256 threads streaming batches of
// systems through LDS (rows are read and written as whole contiguous runs):
//  * cheb_fft: Gauss points and N a power of two (8 .. 2048).  The cosine
//    sums of type II (forward) and III (inverse) come from one complex FFT of
//    length N per system (Makhoul's reordering; the real and imaginary parts
//    of a system ride in one complex sequence and are separated with the
//    X_k / X_{N-k} symmetry), a mixed radix-8/4/2 Stockham FFT through LDS
//    with the twiddles tabulated once per work group.
//  * cheb_direct: any N, Gauss or Gauss-Lobatto points: the cosine sums
//    written out, O(N^2) per system, cosines from an LDS table indexed by the
//    exact integer multiple of the angle.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "shen_launch.hpp"
#include "shen_rows.hpp"

namespace shen {
namespace {

constexpr int kTfThreads = 256;
constexpr int kTfPoints = 2048;  // points per batch in cheb_fft (8 per thread)

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(__builtin_fma(a.x, b.x, -a.y * b.y), __builtin_fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
// -i a (forward sign) or +i a (inverse)
template <bool INV>
__device__ __forceinline__ double2 rot90(double2 a) {
  return INV ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

// In-register DFTs of length 2, 4, 8 with kernel exp(-+2 pi i r k / R).
template <int R, bool INV>
__device__ __forceinline__ void dft(double2 (&v)[R]) {
  if constexpr (R == 2) {
    const double2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    const double2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    const double2 s13 = cadd(v[1], v[3]), d13 = rot90<INV>(csub(v[1], v[3]));
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
  } else {
    // two length-4 DFTs over the even and odd samples, then one radix-2 step
    double2 e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
    dft<4, INV>(e);
    dft<4, INV>(o);
    constexpr double h = 0.70710678118654752440084436210485;  // 1/sqrt(2)
    // o[k] *= exp(-+ 2 pi i k / 8), k = 1, 2, 3
    o[1] = INV ? make_double2(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y))
               : make_double2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
    o[2] = rot90<INV>(o[2]);
    o[3] = INV ? make_double2(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y))
               : make_double2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = cadd(e[k], o[k]);
      v[k + 4] = csub(e[k], o[k]);
    }
  }
}

// LDS slot of point e of the batch: one pad slot per 8 points, so that the
// first pass's writes (stride R points) and every other access (consecutive
// points per 8-lane group) fall in distinct 16-byte bank groups.
__device__ __forceinline__ int lp(int e) { return e + (e >> 3); }
constexpr int kTfSlots = kTfPoints + kTfPoints / 8;

// Radix of pass number `pass` (Ns = product of the earlier radices): 8 while
// at least 8 points per sequence remain, then 4 or 2.
__device__ __host__ __forceinline__ int pass_radix(int N, int Ns) {
  const int left = N / Ns;
  return left >= 8 ? 8 : left;
}

// One Stockham pass of radix R over SB sequences of length N held in buf:
// butterfly j of a sequence reads x[j + r N/R], multiplies by w^(r (j mod Ns))
// with w = exp(-+2 pi i / (Ns R)), transforms, and writes
// y[(j / Ns) Ns R + (j mod Ns) + r Ns].  The pass reads everything into
// registers, waits, then overwrites buf (one buffer, two barriers).
// tw: this pass's twiddles, w^(jm r) at tw[jm (R-1) + r - 1], jm < Ns.
// N, Ns and R are powers of two: lgN = log2 N, lgNs = log2 Ns (index
// arithmetic by shifts and masks).
// ld(base, k): input point k of the sequence at buf offset base (the first
// pass of the inverse forms its inputs on the fly from the raw coefficients).
struct LdsLoad {
  const double2* buf;
  __device__ __forceinline__ double2 operator()(int base, int k) const { return buf[lp(base + k)]; }
};
template <int R, bool INV, typename Load>
__device__ __forceinline__ void fft_pass(double2* buf, const double2* tw, int lgN, int lgNs, int SB, int tid, Load ld) {
  constexpr int PER = 8 / R;  // butterflies per thread (8 points per thread)
  constexpr int lgR = R == 8 ? 3 : (R == 4 ? 2 : 1);
  const int Ns = 1 << lgNs;
  const int lgnb = lgN - lgR;
  const int nb = 1 << lgnb;  // butterflies per sequence
  const int total = SB * nb;
  double2 v[PER][R];
  int dst[PER];
#pragma unroll
  for (int t = 0; t < PER; ++t) {
    const int b = tid + t * kTfThreads;
    dst[t] = -1;
    if (b < total) {
      const int s = b >> lgnb, j = b & (nb - 1);
      const int base = s << lgN;
      const int jm = j & (Ns - 1);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double2 a = ld(base, j + r * nb);
        if (r > 0 && jm > 0) {
          const double2 w = tw[jm * (R - 1) + r - 1];
          a = cmul(a, INV ? cconj(w) : w);
        }
        v[t][r] = a;
      }
      dft<R, INV>(v[t]);
      dst[t] = base + ((j >> lgNs) << (lgNs + lgR)) + jm;
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < PER; ++t) {
    if (dst[t] >= 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[lp(dst[t] + r * Ns)] = v[t][r];
    }
  }
  __syncthreads();
}

// All passes; the first reads its inputs through `first`, the others from buf.
template <bool INV, typename First = LdsLoad>
__device__ __forceinline__ void fft_all(double2* buf, const double2* tw, int lgN, int SB, int tid, First first) {
  const LdsLoad plain{buf};
  int lgNs = 0, off = 0;
  {
    const int left = lgN;  // first pass (lgN >= 3: N >= 8)
    if (left >= 3) {
      fft_pass<8, INV>(buf, tw, lgN, 0, SB, tid, first);
      off = 7;
      lgNs = 3;
    } else if (left == 2) {
      fft_pass<4, INV>(buf, tw, lgN, 0, SB, tid, first);
      off = 3;
      lgNs = 2;
    } else {
      fft_pass<2, INV>(buf, tw, lgN, 0, SB, tid, first);
      off = 1;
      lgNs = 1;
    }
  }
  while (lgNs < lgN) {
    const int left = lgN - lgNs;
    if (left >= 3) {
      fft_pass<8, INV>(buf, tw + off, lgN, lgNs, SB, tid, plain);
      off += 7 << lgNs;
      lgNs += 3;
    } else if (left == 2) {
      fft_pass<4, INV>(buf, tw + off, lgN, lgNs, SB, tid, plain);
      off += 3 << lgNs;
      lgNs += 2;
    } else {
      fft_pass<2, INV>(buf, tw + off, lgN, lgNs, SB, tid, plain);
      off += 1 << lgNs;
      lgNs += 1;
    }
  }
}

// Twiddles of every pass, pass after pass: exp(-2 pi i jm r / (Ns R)) at
// off + jm (R-1) + r - 1 (N - 1 entries in all).
__device__ __forceinline__ void fill_twiddles(double2* tw, int N) {
  int Ns = 1, off = 0;
  while (Ns < N) {
    const int R = pass_radix(N, Ns);
    const int cnt = Ns * (R - 1);
    for (int i = threadIdx.x; i < cnt; i += kTfThreads) {
      const int jm = i / (R - 1), r = i - jm * (R - 1) + 1;
      double sn, cs;
      sincospi(2.0 * (double)(jm * r) / (double)(Ns * R), &sn, &cs);
      tw[off + i] = make_double2(cs, -sn);
    }
    off += cnt;
    Ns *= R;
  }
}

// Shen combination of Chebyshev-type values c (space 1: c_k - c_{k+2};
// space 2: c_k - 2(k+2)/(k+3) c_{k+2} + (k+1)/(k+3) c_{k+4}) at row k of a
// length-N sequence; rows past n read as zero only where the combination
// stays inside 0 .. N-1 (it always does for k < n).
__device__ __forceinline__ double2 shen_combine(const double2* c, int k, int space) {
  if (space == SHEN_SPACE_DIRICHLET) return csub(c[k], c[k + 2]);
  const double K = (double)k;
  const double r = 1.0 / (K + 3.0);  // one division for both weights
  const double g1 = 2.0 * (K + 2.0) * r, g2 = (K + 1.0) * r;
  return c_fma(g2, c[k + 4], c_fma(-g1, c[k + 2], c[k]));
}
// Chebyshev coefficient z_k of sum_j f_j phi_j (the transposed combination),
// f holding n = N-2 or N-4 Shen coefficients (the rest is ignored).
__device__ __forceinline__ double2 shen_to_cheb(const double2* f, int k, int n, int space) {
  if (space == SHEN_SPACE_CHEBYSHEV) return f[k];
  double2 z = k < n ? f[k] : zero2();
  if (space == SHEN_SPACE_DIRICHLET) return (k >= 2 && k - 2 < n) ? csub(z, f[k - 2]) : z;
  // weights -2k/(k+1) of f_{k-2} and (k-3)/(k-1) of f_{k-4}, from one
  // division: 1/(k+1) = (k-1) R and 1/(k-1) = (k+1) R with R = 1/((k+1)(k-1))
  const double K = (double)k;
  const double R = 1.0 / ((K + 1.0) * (K - 1.0));
  if (k >= 2 && k - 2 < n) z = c_fma(-2.0 * K * ((K - 1.0) * R), f[k - 2], z);
  if (k >= 4 && k - 4 < n) z = c_fma((K - 3.0) * ((K + 1.0) * R), f[k - 4], z);
  return z;
}
__device__ __forceinline__ int space_n(int space, int N) {
  return space == SHEN_SPACE_CHEBYSHEV ? N : (space == SHEN_SPACE_DIRICHLET ? N - 2 : N - 4);
}

// Output of the forward direction at row k from the Chebyshev scalar
// products c (already weighted): the space's scalar product, or for the
// Chebyshev space with `solve` the coefficient c_k / (c_k' pi / 2).
__device__ __forceinline__ double2 forward_out(const double2* c, int k, int N, int space, int solve, int gl) {
  const int n = space_n(space, N);
  if (k >= n) return zero2();
  if (space == SHEN_SPACE_CHEBYSHEV) {
    if (!solve) return c[k];
    const double ckk = (k == 0 || (gl && k == N - 1)) ? 2.0 : 1.0;
    return cscale(2.0 / (ckk * kPi), c[k]);
  }
  return shen_combine(c, k, space);
}

// Dirichlet mass solve B u = s of every parity chain of a batch, in place in
// LDS.  At Gauss points B is, per chain, tridiagonal with off-diagonals -pi/2
// and diagonal pi, except 3 pi / 2 in row 0 (c_0 = 2), so its LU pivots have
// a closed form: d_m = (pi/2) r_m with r_m = (2m+3)/(2m+1) (even chain) or
// (m+2)/(m+1) (odd chain) at chain row m (r_{m+1} = 2 - 1/r_m).  Forward
// y_m = s_m + a_m y_{m-1} with a_m = (pi/2) / d_{m-1}, then backward
// u_m = b_m + e_m u_{m+1} with b_m = y_m / d_m, e_m = (pi/2) / d_m.
// T = N/16 lanes per chain, 8 chain rows each (a chain has at most N/2 rows);
// every first-order recurrence is solved per lane from a zero carry, the
// lanes' affine maps (product of the coefficients, local result) are
// scanned across the chain's lanes with shuffles, and the carry is added
// back.  T divides 64, so a chain's lanes sit in one wavefront.
__device__ __forceinline__ double dirichlet_rpivot(int p, int m) {  // 1 / d_m
  const double M = (double)m;
  return p == 0 ? (2.0 / kPi) * (2.0 * M + 1.0) * fast_rcp(2.0 * M + 3.0)
                : (2.0 / kPi) * (M + 1.0) * fast_rcp(M + 2.0);
}
__device__ __forceinline__ void dirichlet_mass_lanes(double2* buf, int tid, int lgN, int n, int sb) {
  const int T = 1 << (lgN - 4);              // lanes per chain
  const int ch = tid >> (lgN - 4), q = tid & (T - 1);
  const int s = ch >> 1, p = ch & 1;
  const bool act = s < sb;
  const int nm = (n - p + 1) / 2;            // rows of this chain
  const int base = s << lgN;
  const double c = 0.5 * kPi;
  // 1/d of rows 8q - 1 .. 8q + 7 (0 outside the chain); a_m = c rd_{m-1},
  // e_m = c rd_m (so a is 0 at row 0 and past the chain, e past it)
  double rd[9];
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    const int m = 8 * q + j - 1;
    rd[j] = (m >= 0 && m < nm) ? dirichlet_rpivot(p, m) : 0.0;
  }
  auto a_of = [&](int j) { return 8 * q + j < nm ? c * rd[j] : 0.0; };
  auto e_of = [&](int j) { return c * rd[j + 1]; };
  double2 v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int m = 8 * q + j;
    v[j] = (act && m < nm) ? buf[lp(base + 2 * m + p)] : zero2();
  }
  // forward: local sweep from a zero carry; P = product of the a's
  double P = 1.0;
  double2 y = zero2();
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const double am = a_of(j);
    y = c_fma(am, y, v[j]);
    v[j] = y;
    P *= am;
  }
  // exclusive scan over the lanes of the chain: carry into lane q
  double cP = P;
  double2 cy = y;
  for (int d = 1; d < T; d <<= 1) {
    const double oP = __shfl_up(cP, d, T);
    const double2 oy = make_double2(__shfl_up(cy.x, d, T), __shfl_up(cy.y, d, T));
    if (q >= d) {
      cy = c_fma(cP, oy, cy);
      cP *= oP;
    }
  }
  double2 yin = make_double2(__shfl_up(cy.x, 1, T), __shfl_up(cy.y, 1, T));
  if (q == 0) yin = zero2();
  double pj = 1.0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    pj *= a_of(j);
    v[j] = c_fma(pj, yin, v[j]);
  }
  // backward: u_m = (y_m + c u_{m+1}) / d_m, local from a zero carry
  double E = 1.0;
  double2 x = zero2();
#pragma unroll
  for (int j = 7; j >= 0; --j) {
    const double rdm = rd[j + 1];  // (0 past the chain)
    x = cscale(rdm, c_fma(c, x, v[j]));
    v[j] = x;
    E *= c * rdm;
  }
  // inclusive suffix scan: carry into lane q from the lanes above it
  double cE = E;
  double2 cx = x;
  for (int d = 1; d < T; d <<= 1) {
    const double oE = __shfl_down(cE, d, T);
    const double2 ox = make_double2(__shfl_down(cx.x, d, T), __shfl_down(cx.y, d, T));
    if (q + d < T) {
      cx = c_fma(cE, ox, cx);
      cE *= oE;
    }
  }
  double2 xin = make_double2(__shfl_down(cx.x, 1, T), __shfl_down(cx.y, 1, T));
  if (q == T - 1) xin = zero2();
  double ej = 1.0;
#pragma unroll
  for (int j = 7; j >= 0; --j) {
    const int m = 8 * q + j;
    ej *= e_of(j);
    if (act && m < nm) buf[lp(base + 2 * m + p)] = c_fma(ej, xin, v[j]);
  }
}

// ---------------------------------------------------------------- FFT path
// dir 0: point values -> scalar products (with solve: the coefficients, i.e.
// for the Chebyshev space the scaled products, for the Dirichlet space the
// mass solve of dirichlet_mass_lanes in LDS: the whole forward transform in one
// pass); dir 1: Shen coefficients -> point values.  Gauss points, N = 2^m.
// Each thread moves 8 points of a batch; the next batch's rows are loaded
// into registers while the current one is transformed.
// Three work groups per CU (LDS allows three at N = 512): the inverse is held
// to the forward's register budget for that.
// MASS (a separate instance, so that the others keep their registers): the
// Dirichlet forward transform, with the mass solve after the scalar products.
template <int DIR, bool MASS = false>
__global__ __launch_bounds__(kTfThreads, (MASS ? 2 : 3)) void cheb_fft(int N, int64_t nsys, int space, int solve,
                                                       const double2* __restrict__ in, double2* __restrict__ out) {
  constexpr int dir = DIR;
  extern __shared__ double2 lds[];
  constexpr int PT = kTfPoints / kTfThreads;  // points per thread
  double2* buf = lds;                         // kTfSlots (padded points)
  double2* tw = lds + kTfSlots;               // N - 1 pass twiddles (+1 spare)
  double2* wq = tw + N;                       // N: exp(-i pi k / (2N))
  const int SB = kTfPoints / N;               // N <= kTfPoints, a power of two
  const int lgN = 31 - __builtin_clz(N);
  fill_twiddles(tw, N);
  for (int q = threadIdx.x; q < N; q += kTfThreads) {
    double sn, cs;
    sincospi((double)q / (2.0 * (double)N), &sn, &cs);
    wq[q] = make_double2(cs, -sn);
  }
  const int64_t nbatch = (nsys + SB - 1) / SB;
  const int n = space_n(space, N);
  const double wsc = 0.5 * kPi / (double)N;
  // rows of batch bt into registers (point i = threadIdx.x + t * kTfThreads)
  double2 nx[PT];
  auto load = [&](int64_t bt, int tid) {
    const int64_t w0 = bt * SB;
#pragma unroll
    for (int t = 0; t < PT; ++t) {
      const int i = tid + t * kTfThreads;
      const int s = i >> lgN, k = i & (N - 1);
      const bool ok = w0 + s < nsys && (dir == 0 || k < n);
      nx[t] = ok ? in[(w0 + s) * (int64_t)N + k] : zero2();
    }
  };
  int64_t bt = blockIdx.x;
  if (bt < nbatch) load(bt, threadIdx.x);
  for (; bt < nbatch; bt += gridDim.x) {
    // the thread index is re-derived every batch from an opaque copy, so that
    // the per-point constants (indices, combination weights) are not hoisted
    // out of the loop and held in registers across it
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    tid &= kTfThreads - 1;
    const int64_t w0 = bt * SB;
    const int sb = (int)((nsys - w0) < SB ? (nsys - w0) : SB);
    __syncthreads();  // the previous batch is out of buf (and the tables are in)
    if constexpr (dir == 0) {
      // Makhoul's reordering: v_q = u_{2q}, v_{N-1-q} = u_{2q+1}
#pragma unroll
      for (int t = 0; t < PT; ++t) {
        const int i = tid + t * kTfThreads;
        const int s = i >> lgN, j = i & (N - 1);
        const int q = (j & 1) ? N - 1 - (j >> 1) : (j >> 1);
        buf[lp((s << lgN) + q)] = nx[t];
      }
    } else {
#pragma unroll
      for (int t = 0; t < PT; ++t) buf[lp(tid + t * kTfThreads)] = nx[t];
    }
    if (bt + gridDim.x < nbatch) load(bt + gridDim.x, tid);
    __syncthreads();
    double2 cv[PT];
    if constexpr (dir == 0) {
      fft_all<false>(buf, tw, lgN, SB, tid, LdsLoad{buf});
      // C_k = (W_k V_k + conj(W_k) V_{N-k}) / 2 times the Gauss weight pi/N,
      // formed where the space's combination needs it (rows k, k+2, k+4)
      auto cheb = [&](int s, int k) {
        const double2 Vk = buf[lp((s << lgN) + k)], Vm = buf[lp((s << lgN) + ((N - k) & (N - 1)))];
        const double2 W = wq[k];
        return cscale(wsc, cadd(cmul(W, Vk), cmul(cconj(W), Vm)));
      };
#pragma unroll
      for (int t = 0; t < PT; ++t) {
        const int i = tid + t * kTfThreads;
        const int s = i >> lgN, k = i & (N - 1);
        double2 r = zero2();
        if (k < n) {
          if (space == SHEN_SPACE_CHEBYSHEV) {
            r = cheb(s, k);
            if (solve) r = cscale(2.0 / ((k == 0 ? 2.0 : 1.0) * kPi), r);
          } else if (space == SHEN_SPACE_DIRICHLET) {
            r = csub(cheb(s, k), cheb(s, k + 2));
          } else {
            const double K = (double)k, r3 = fast_rcp(K + 3.0);
            r = c_fma((K + 1.0) * r3, cheb(s, k + 4), c_fma(-2.0 * (K + 2.0) * r3, cheb(s, k + 2), cheb(s, k)));
          }
        }
        cv[t] = r;
      }
      if constexpr (MASS) {
        // the forward transform: the mass solve of every chain of the batch
        // in LDS (one thread per chain), before the batch goes out
        __syncthreads();  // every read of the FFT output is done
#pragma unroll
        for (int t = 0; t < PT; ++t) buf[lp(tid + t * kTfThreads)] = cv[t];
        __syncthreads();
        dirichlet_mass_lanes(buf, tid, lgN, n, sb);
        __syncthreads();
#pragma unroll
        for (int t = 0; t < PT; ++t) cv[t] = buf[lp(tid + t * kTfThreads)];
      }
#pragma unroll
      for (int t = 0; t < PT; ++t) {
        const int i = tid + t * kTfThreads;
        const int s = i >> lgN, k = i & (N - 1);
        if (s < sb) out[(w0 + s) * (int64_t)N + k] = cv[t];
      }
    } else {
      // Shen -> Chebyshev coefficients z (the transposed combination), then
      // V_k = exp(i pi k / (2N)) (Z_k - i Z_{N-k}) with Z_0 = z_0, Z_k = z_k / 2
      auto zc = [&](int s, int k) {
        const int i = (s << lgN) + k;
        double2 z;
        if (space == SHEN_SPACE_CHEBYSHEV) {
          z = buf[lp(i)];
        } else {
          z = k < n ? buf[lp(i)] : zero2();
          if (space == SHEN_SPACE_DIRICHLET) {
            if (k >= 2 && k - 2 < n) z = csub(z, buf[lp(i - 2)]);
          } else {
            // weights -2k/(k+1) and (k-3)/(k-1) from one reciprocal (as shen_to_cheb)
            const double K = (double)k;
            const double R = fast_rcp((K + 1.0) * (K - 1.0));
            if (k >= 2 && k - 2 < n) z = c_fma(-2.0 * K * ((K - 1.0) * R), buf[lp(i - 2)], z);
            if (k >= 4 && k - 4 < n) z = c_fma((K - 3.0) * ((K + 1.0) * R), buf[lp(i - 4)], z);
          }
        }
        return k == 0 ? z : cscale(0.5, z);
      };
      // formed by the first FFT pass as it reads its inputs (buf still holds
      // the raw coefficients then; the pass writes only after its barrier)
      auto pre = [&](int base, int k) {
        const int s = base >> lgN;
        const double2 Zk = zc(s, k);
        const double2 Zm = k == 0 ? zero2() : zc(s, N - k);
        const double2 d = make_double2(Zk.x + Zm.y, Zk.y - Zm.x);  // Z_k - i Z_{N-k}
        return cmul(cconj(wq[k]), d);
      };
      fft_all<true>(buf, tw, lgN, SB, tid, pre);
      // u_{2q} = v_q, u_{2q+1} = v_{N-1-q}
#pragma unroll
      for (int t = 0; t < PT; ++t) {
        const int i = tid + t * kTfThreads;
        const int s = i >> lgN, j = i & (N - 1);
        const int q = (j & 1) ? N - 1 - (j >> 1) : (j >> 1);
        cv[t] = buf[lp((s << lgN) + q)];
      }
#pragma unroll
      for (int t = 0; t < PT; ++t) {
        const int i = tid + t * kTfThreads;
        const int s = i >> lgN, j = i & (N - 1);
        if (s < sb) out[(w0 + s) * (int64_t)N + j] = cv[t];
      }
    }
  }
}

// ------------------------------------------------------------- direct path
// Any N, Gauss (gl = 0) or Gauss-Lobatto (gl = 1) points.  cosines
// cos(pi q / M) for q < 2M: M = 2N (Gauss: angle pi k (2j+1) / (2N)),
// M = N-1 (Gauss-Lobatto: angle pi k j / (N-1)).
__global__ __launch_bounds__(kTfThreads) void cheb_direct(int N, int64_t nsys, int space, int dir, int solve, int gl, int SB,
                                                          const double2* __restrict__ in, double2* __restrict__ out) {
  extern __shared__ double2 lds[];
  const int M = gl ? (N > 1 ? N - 1 : 1) : 2 * N;
  double* ct = reinterpret_cast<double*>(lds);  // 2M cosines (padded to an even count)
  double2* buf = lds + M;                        // SB N inputs
  double2* res = buf + SB * N;                   // SB N results
  for (int q = threadIdx.x; q < 2 * M; q += kTfThreads) ct[q] = cospi((double)q / (double)M);
  __syncthreads();
  const int64_t nbatch = (nsys + SB - 1) / SB;
  const int P = SB * N;
  const int n = space_n(space, N);
  const double wgc = kPi / (double)N, wgl = N > 1 ? kPi / (double)(N - 1) : kPi;
  for (int64_t bt = blockIdx.x; bt < nbatch; bt += gridDim.x) {
    const int64_t w0 = bt * SB;
    const int sb = (int)((nsys - w0) < SB ? (nsys - w0) : SB);
    for (int i = threadIdx.x; i < P; i += kTfThreads) {
      const int s = i / N, k = i - s * N;
      const bool ok = s < sb && (dir == 0 || k < n);
      buf[i] = ok ? in[(w0 + s) * (int64_t)N + k] : zero2();
    }
    __syncthreads();
    if (dir == 1) {
      // Shen -> Chebyshev coefficients into res, then back into buf
      for (int i = threadIdx.x; i < P; i += kTfThreads) {
        const int s = i / N, k = i - s * N;
        res[i] = shen_to_cheb(buf + s * N, k, n, space);
      }
      __syncthreads();
      for (int i = threadIdx.x; i < P; i += kTfThreads) buf[i] = res[i];
      __syncthreads();
    }
    // cosine sums: forward C_k = sum_j u_j cos(.) sigma_j, inverse u_j = sum_k z_k cos(.)
    for (int i = threadIdx.x; i < P; i += kTfThreads) {
      const int s = i / N, r = i - s * N;  // r: output row (k forward, j inverse)
      const double2* x = buf + s * N;
      double2 acc = zero2();
      int q = 0;
      // q advances by the multiplier of the summation index, modulo 2M
      const int mult = gl ? r : (dir == 0 ? 2 * r : 2 * r + 1);
      const int q0 = gl ? 0 : (dir == 0 ? r : 0);
      q = q0 % (2 * M);
      const int dq = mult % (2 * M);
      for (int m = 0; m < N; ++m) {
        double c = ct[q];
        if (dir == 0) c *= gl ? ((m == 0 || m == N - 1) ? 0.5 * wgl : wgl) : wgc;
        acc = c_fma(c, x[m], acc);
        q += dq;
        if (q >= 2 * M) q -= 2 * M;
      }
      res[i] = acc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < P; i += kTfThreads) {
      const int s = i / N, k = i - s * N;
      if (s < sb) out[(w0 + s) * (int64_t)N + k] = dir == 0 ? forward_out(res + s * N, k, N, space, solve, gl) : res[i];
    }
    __syncthreads();
  }
}

int grid_for(const void* kernel, int64_t batches, size_t lds) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kTfThreads, lds) != hipSuccess || per_cu < 1) per_cu = 1;
  const int64_t slots = (int64_t)cus * per_cu;
  return (int)(batches < slots ? (batches > 0 ? batches : 1) : slots);
}

}  // namespace

bool transform_fft_ok(int N, int gl) { return !gl && N >= 8 && N <= kTfPoints && (N & (N - 1)) == 0; }
// The Dirichlet forward transform in one pass (FFT kernel with the mass solve
// of dirichlet_mass_lanes): a chain's N/16 lanes within one wavefront.
bool transform_fused_mass_ok(int N, int gl) { return transform_fft_ok(N, gl) && N >= 16 && N <= 1024; }

size_t transform_direct_lds(int N, int gl, int* sb_out) {
  const int M = gl ? (N > 1 ? N - 1 : 1) : 2 * N;
  int SB = 4096 / N;
  if (SB < 1) SB = 1;
  if (SB > 64) SB = 64;
  if (sb_out) *sb_out = SB;
  return (size_t)M * sizeof(double2) + (size_t)2 * SB * N * sizeof(double2);
}

hipError_t launch_transform(int N, int64_t nsys, int space, int dir, int solve, int gl, const void* in, void* out,
                            void* stream) {
  if (nsys <= 0) return hipSuccess;
  hipStream_t st = (hipStream_t)stream;
  if (transform_fft_ok(N, gl)) {
    const size_t lds = (size_t)(kTfSlots + 2 * N) * sizeof(double2);
    static const bool attr =
        hipFuncSetAttribute((const void*)cheb_fft<0>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) == hipSuccess &&
        hipFuncSetAttribute((const void*)cheb_fft<0, true>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) ==
            hipSuccess &&
        hipFuncSetAttribute((const void*)cheb_fft<1>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) == hipSuccess;
    (void)attr;
    const int SB = kTfPoints / N;
    const int64_t batches = (nsys + SB - 1) / SB;
    const bool mass = dir == 0 && solve && space == SHEN_SPACE_DIRICHLET && transform_fused_mass_ok(N, gl);
    const void* k = mass ? (const void*)cheb_fft<0, true> : dir == 0 ? (const void*)cheb_fft<0> : (const void*)cheb_fft<1>;
    const int grid = grid_for(k, batches, lds);
    if (mass)
      hipLaunchKernelGGL((cheb_fft<0, true>), dim3((unsigned)grid), dim3(kTfThreads), lds, st, N, nsys, space, solve,
                         (const double2*)in, (double2*)out);
    else if (dir == 0)
      hipLaunchKernelGGL(cheb_fft<0>, dim3((unsigned)grid), dim3(kTfThreads), lds, st, N, nsys, space, solve,
                         (const double2*)in, (double2*)out);
    else
      hipLaunchKernelGGL(cheb_fft<1>, dim3((unsigned)grid), dim3(kTfThreads), lds, st, N, nsys, space, solve,
                         (const double2*)in, (double2*)out);
    return hipGetLastError();
  }
  int SB = 1;
  const size_t lds = transform_direct_lds(N, gl, &SB);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  static const bool attr =
      hipFuncSetAttribute((const void*)cheb_direct, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) == hipSuccess;
  (void)attr;
  const int64_t batches = (nsys + SB - 1) / SB;
  const int grid = grid_for((const void*)cheb_direct, batches, lds);
  hipLaunchKernelGGL(cheb_direct, dim3((unsigned)grid), dim3(kTfThreads), lds, st, N, nsys, space, dir, solve, gl, SB,
                     (const double2*)in, (double2*)out);
  return hipGetLastError();
}

}  // namespace shen
