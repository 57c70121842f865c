// Host-side launch interface shared by the C-ABI layer and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "shenhip.h"

namespace shen {

enum class ChainKind { HelmSolve, HelmAdjoint, HelmMatvec, HelmMixed, BihSolve, BihAdjoint, BihMatvec, BihMixed };

struct ChainArgs {
  ChainKind kind;
  int N = 0;
  int64_t nsys = 0;
  const double* c0 = nullptr;  // alpha or a
  const double* c1 = nullptr;  // b
  const void* f = nullptr;     // input rows (f, gbar or u)
  void* u = nullptr;           // output rows (u, lambda or Hu)
  const void* ufwd = nullptr;  // adjoint: forward solution (for coefficient gradients)
  double* g0 = nullptr;        // adjoint: grad alpha / grad a
  double* g1 = nullptr;        // adjoint: grad b
  int32_t* info = nullptr;
  int32_t* iters = nullptr;  // mixed: corrections applied per system
  int gl = 0;
  int trans = 0;
  int it_max = 8;
  double tol = 1e-14;
  size_t lds_budget = 65536;
  void* stream = nullptr;
  // matvec kernels: Crank-Nicolson right-hand side instead of H u (see RhsTerms)
  int rhs = 0;
  double inv = 0.0;
  double sigma = 0.0;
  const void* sh = nullptr;
};

struct WaveArgs {
  int family = 0;  // 0 Helmholtz, 1 biharmonic
  int N = 0;
  int64_t nsys = 0;
  const double* c0 = nullptr;
  const double* c1 = nullptr;
  const void* f = nullptr;
  void* u = nullptr;  // must not alias f (restart states are parked in it)
  int32_t* info = nullptr;
  int32_t* iters = nullptr;  // mixed: corrections applied per system
  int gl = 0;
  int chunk = 0;   // preferred chunk length C (0: automatic)
  int mixed = 0;   // FP32 factor/solve + FP64 refinement
  int it_max = 8;  // refinement steps at most
  double tol = 1e-14;
  // adjoint: f = gbar, u = lambda (must not alias gbar); ufwd = forward
  // solution and g0/g1 = coefficient gradients (optional)
  int adjoint = 0;
  const void* ufwd = nullptr;
  double* g0 = nullptr;
  double* g1 = nullptr;
  void* stream = nullptr;
  // factor-once mode: fac holds the restart states, [nsys][2 G NS] double2
  // (NS = 1 Helmholtz, 5 biharmonic).  fac_mode 1: only the boundary walk,
  // into fac; 2: only the wave solve, states from fac (u may alias f).
  void* fac = nullptr;
  int fac_mode = 0;
  // mass solves (family 0 only): right-hand side Cbar f instead of f
  int deriv = 0;
  // matvec kernels: Crank-Nicolson right-hand side sigma S(h) - H' u, where c0
  // holds K2 per system and H' is the system matrix at the coefficients the
  // step maps K2 and inv = 2/(nu dt) to; sh = S(h) rows or null
  int rhs = 0;
  double inv = 0.0;
  double sigma = 0.0;
  const void* sh = nullptr;
};

struct WaveCfg {
  int C, G;
};
__host__ __device__ WaveCfg pick_cfg(int nc, int family, int N, int prefC);
bool wave_supported(int family, int N);
// Large N (chains across wavefronts): wavefronts per work group, 0 if
// (family, N) is not served there; *one (if given): one parity chain per work
// group (N past 4096).  Plain FP64 forward solves out of place only.
int multi_waves(int family, int N, bool* one = nullptr);
hipError_t launch_multi(const WaveArgs& a);
bool wave_chunk_ok(int family, int N, int chunk);
// Batched form: the host descriptors (validated, planned), one launch pair
// per class; `work` holds batched_counters(ndesc) queue counters.
// fork: deal the classes to side streams forked from and joined to `stream`
// (false: everything in order on `stream`, creating nothing).
hipError_t launch_batched(const shen_problem* desc, int ndesc, void* work, int gl, void* stream, bool fork);
// Creates the current device's side streams of launch_batched now (a planning
// call), so that a solve under graph capture creates nothing.
hipError_t batched_fork_prepare();
int batched_counters(int ndesc);
// Library-owned counter array of the batched launch (one per device, 8-byte
// words): device address for the current device, looked up on first use.
constexpr int kBatchedStaticWords = 512;
constexpr int kMaxDevices = 64;
hipError_t batched_static_scratch(void** ptr);
hipError_t launch_wave(const WaveArgs& a);
int64_t wave_state_slot(int family, int N, int chunk);
bool matvec_wave_supported(int family, int N);
hipError_t launch_matvec_wave(const WaveArgs& a);
bool mass_wave_supported(int N);
hipError_t launch_mass_wave(const WaveArgs& a);  // family, N, nsys, f, u (may alias f), gl, stream

// Shen transforms: dir 0 point values -> scalar products (solve: Chebyshev
// coefficients), dir 1 Shen coefficients -> point values
bool transform_fft_ok(int N, int gl);
bool transform_fused_mass_ok(int N, int gl);
size_t transform_direct_lds(int N, int gl, int* sb_out);
hipError_t launch_transform(int N, int64_t nsys, int space, int dir, int solve, int gl, const void* in, void* out,
                            void* stream);

size_t chain_bytes_per_system(ChainKind kind, int N);
int chain_systems_per_block(ChainKind kind, int N, size_t lds_budget);
hipError_t launch_chain(const ChainArgs& a);

}  // namespace shen
