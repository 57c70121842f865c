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
__device__ __forceinline__ void dft(double2 (&v)[8]) {
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
    double2 e[8] = {v[0], v[2], v[4], v[6]}, o[8] = {v[1], v[3], v[5], v[7]};
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

// One Stockham pass of radix R over SB sequences of length N held in buf:
// butterfly j of a sequence reads x[j + r N/R], multiplies by w^(r (j mod Ns))
// with w = exp(-+2 pi i / (Ns R)), transforms, and writes
// y[(j / Ns) Ns R + (j mod Ns) + r Ns].  The pass reads everything into
// registers, waits, then overwrites buf (one buffer, two barriers).
// tw[q] = exp(-2 pi i q / N), q < N.
template <int R, bool INV>
__device__ __forceinline__ void fft_pass(double2* buf, const double2* tw, int N, int Ns, int SB) {
  constexpr int PER = 8 / R;  // butterflies per thread (8 points per thread)
  const int nb = N / R;       // butterflies per sequence
  const int total = SB * nb;
  double2 v[PER][8];
  int dst[PER];
#pragma unroll
  for (int t = 0; t < PER; ++t) {
    const int b = threadIdx.x + t * kTfThreads;
    dst[t] = -1;
    if (b < total) {
      const int s = b / nb, j = b - s * nb;
      double2* x = buf + s * N;
      const int jm = j % Ns;
      const int step = (N / (Ns * R)) * jm;  // twiddle index step per r
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double2 a = x[j + r * nb];
        if (r > 0 && jm > 0) {
          const double2 w = tw[(step * r) & (N - 1)];
          a = cmul(a, INV ? cconj(w) : w);
        }
        v[t][r] = a;
      }
      dft<R, INV>(v[t]);
      dst[t] = s * N + (j / Ns) * Ns * R + jm;
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < PER; ++t) {
    if (dst[t] >= 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) buf[dst[t] + r * Ns] = v[t][r];
    }
  }
  __syncthreads();
}

template <bool INV>
__device__ __forceinline__ void fft_all(double2* buf, const double2* tw, int N, int SB) {
  int Ns = 1;
  while (Ns < N) {
    const int left = N / Ns;
    if (left >= 8) {
      fft_pass<8, INV>(buf, tw, N, Ns, SB);
      Ns *= 8;
    } else if (left == 4) {
      fft_pass<4, INV>(buf, tw, N, Ns, SB);
      Ns *= 4;
    } else {
      fft_pass<2, INV>(buf, tw, N, Ns, SB);
      Ns *= 2;
    }
  }
}

// Shen combination of Chebyshev-type values c (space 1: c_k - c_{k+2};
// space 2: c_k - 2(k+2)/(k+3) c_{k+2} + (k+1)/(k+3) c_{k+4}) at row k of a
// length-N sequence; rows past n read as zero only where the combination
// stays inside 0 .. N-1 (it always does for k < n).
__device__ __forceinline__ double2 shen_combine(const double2* c, int k, int space) {
  if (space == SHEN_SPACE_DIRICHLET) return csub(c[k], c[k + 2]);
  const double K = (double)k;
  const double g1 = 2.0 * (K + 2.0) / (K + 3.0), g2 = (K + 1.0) / (K + 3.0);
  return c_fma(g2, c[k + 4], c_fma(-g1, c[k + 2], c[k]));
}
// Chebyshev coefficient z_k of sum_j f_j phi_j (the transposed combination),
// f holding n = N-2 or N-4 Shen coefficients (the rest is ignored).
__device__ __forceinline__ double2 shen_to_cheb(const double2* f, int k, int n, int space) {
  if (space == SHEN_SPACE_CHEBYSHEV) return f[k];
  double2 z = k < n ? f[k] : zero2();
  if (space == SHEN_SPACE_DIRICHLET) return (k >= 2 && k - 2 < n) ? csub(z, f[k - 2]) : z;
  if (k >= 2 && k - 2 < n) {
    const double K = (double)(k - 2);
    z = c_fma(-2.0 * (K + 2.0) / (K + 3.0), f[k - 2], z);
  }
  if (k >= 4 && k - 4 < n) {
    const double K = (double)(k - 4);
    z = c_fma((K + 1.0) / (K + 3.0), f[k - 4], z);
  }
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

// ---------------------------------------------------------------- FFT path
// dir 0: point values -> scalar products (or Chebyshev coefficients with
// solve); dir 1: Shen coefficients -> point values.  Gauss points, N = 2^m.
__global__ __launch_bounds__(kTfThreads) void cheb_fft(int N, int64_t nsys, int space, int dir, int solve,
                                                       const double2* __restrict__ in, double2* __restrict__ out) {
  extern __shared__ double2 lds[];
  double2* buf = lds;                 // kTfPoints
  double2* tw = lds + kTfPoints;      // N: exp(-2 pi i q / N)
  double2* wq = tw + N;               // N: exp(-i pi k / (2N))
  const int SB = kTfPoints / N < 1 ? 1 : kTfPoints / N;
  for (int q = threadIdx.x; q < N; q += kTfThreads) {
    double s, c;
    sincospi(2.0 * (double)q / (double)N, &s, &c);
    tw[q] = make_double2(c, -s);
    sincospi((double)q / (2.0 * (double)N), &s, &c);
    wq[q] = make_double2(c, -s);
  }
  __syncthreads();
  const int64_t nbatch = (nsys + SB - 1) / SB;
  const int P = SB * N;
  const int n = space_n(space, N);
  for (int64_t bt = blockIdx.x; bt < nbatch; bt += gridDim.x) {
    const int64_t w0 = bt * SB;
    const int sb = (int)((nsys - w0) < SB ? (nsys - w0) : SB);
    if (dir == 0) {
      // load with Makhoul's reordering: v_q = u_{2q}, v_{N-1-q} = u_{2q+1}
      for (int i = threadIdx.x; i < P; i += kTfThreads) {
        const int s = i / N, j = i - s * N;
        const int q = (j & 1) ? N - 1 - (j >> 1) : (j >> 1);
        buf[s * N + q] = s < sb ? in[(w0 + s) * (int64_t)N + j] : zero2();
      }
      __syncthreads();
      fft_all<false>(buf, tw, N, SB);
      // C_k = (W_k V_k + conj(W_k) V_{N-k}) / 2 times the Gauss weight pi/N
      double2 cv[kTfPoints / kTfThreads];
#pragma unroll
      for (int t = 0; t < kTfPoints / kTfThreads; ++t) {
        const int i = threadIdx.x + t * kTfThreads;
        if (i < P) {
          const int s = i / N, k = i - s * N;
          const double2 Vk = buf[s * N + k], Vm = buf[s * N + ((N - k) & (N - 1))];
          const double2 W = wq[k];
          cv[t] = cscale(0.5 * kPi / (double)N, cadd(cmul(W, Vk), cmul(cconj(W), Vm)));
        }
      }
      __syncthreads();
#pragma unroll
      for (int t = 0; t < kTfPoints / kTfThreads; ++t) {
        const int i = threadIdx.x + t * kTfThreads;
        if (i < P) buf[i] = cv[t];
      }
      __syncthreads();
      for (int i = threadIdx.x; i < P; i += kTfThreads) {
        const int s = i / N, k = i - s * N;
        if (s < sb) out[(w0 + s) * (int64_t)N + k] = forward_out(buf + s * N, k, N, space, solve, 0);
      }
    } else {
      // Shen coefficients in, Chebyshev coefficients z, then
      // V_k = exp(i pi k / (2N)) (Z_k - i Z_{N-k}) with Z_0 = z_0, Z_k = z_k / 2
      for (int i = threadIdx.x; i < P; i += kTfThreads) {
        const int s = i / N, k = i - s * N;
        buf[i] = (s < sb && k < n) ? in[(w0 + s) * (int64_t)N + k] : zero2();
      }
      __syncthreads();
      double2 zv[kTfPoints / kTfThreads];
#pragma unroll
      for (int t = 0; t < kTfPoints / kTfThreads; ++t) {
        const int i = threadIdx.x + t * kTfThreads;
        if (i < P) {
          const int s = i / N, k = i - s * N;
          const double2 z = shen_to_cheb(buf + s * N, k, n, space);
          zv[t] = k == 0 ? z : cscale(0.5, z);
        }
      }
      __syncthreads();
#pragma unroll
      for (int t = 0; t < kTfPoints / kTfThreads; ++t) {
        const int i = threadIdx.x + t * kTfThreads;
        if (i < P) buf[i] = zv[t];
      }
      __syncthreads();
#pragma unroll
      for (int t = 0; t < kTfPoints / kTfThreads; ++t) {
        const int i = threadIdx.x + t * kTfThreads;
        if (i < P) {
          const int s = i / N, k = i - s * N;
          const double2 Zm = k == 0 ? zero2() : buf[s * N + (N - k)];
          const double2 d = make_double2(buf[i].x + Zm.y, buf[i].y - Zm.x);  // Z_k - i Z_{N-k}
          zv[t] = cmul(cconj(wq[k]), d);
        }
      }
      __syncthreads();
#pragma unroll
      for (int t = 0; t < kTfPoints / kTfThreads; ++t) {
        const int i = threadIdx.x + t * kTfThreads;
        if (i < P) buf[i] = zv[t];
      }
      __syncthreads();
      fft_all<true>(buf, tw, N, SB);
      // u_{2q} = v_q, u_{2q+1} = v_{N-1-q}
      for (int i = threadIdx.x; i < P; i += kTfThreads) {
        const int s = i / N, j = i - s * N;
        const int q = (j & 1) ? N - 1 - (j >> 1) : (j >> 1);
        if (s < sb) out[(w0 + s) * (int64_t)N + j] = buf[s * N + q];
      }
    }
    __syncthreads();
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
    const size_t lds = (size_t)(kTfPoints + 2 * N) * sizeof(double2);
    static const bool attr =
        hipFuncSetAttribute((const void*)cheb_fft, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) == hipSuccess;
    (void)attr;
    const int SB = kTfPoints / N;
    const int64_t batches = (nsys + SB - 1) / SB;
    const int grid = grid_for((const void*)cheb_fft, batches, lds);
    hipLaunchKernelGGL(cheb_fft, dim3((unsigned)grid), dim3(kTfThreads), lds, st, N, nsys, space, dir, solve,
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
