// C-ABI layer: argument validation, kernel selection, launch on the caller's
// stream.  See include/shenhip.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <cmath>
#include <stdint.h>
#include <string.h>

#include <atomic>
#include <mutex>

#include "shen_launch.hpp"
#include "shenhip.h"

namespace {

using shen::ChainArgs;
using shen::ChainKind;

struct DevInfo {
  size_t lds_max = 0;  // max dynamic LDS per workgroup
  int ok = 0;
};

constexpr int kMaxDevices = 64;
DevInfo g_dev[kMaxDevices];
std::mutex g_dev_mu;

// Fills the per-device table on first use.  Returns SHEN_OK or SHEN_EDEVICE.
int device_info(DevInfo* out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SHEN_EDEVICE;
  std::lock_guard<std::mutex> lock(g_dev_mu);
  if (!g_dev[dev].ok) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) return SHEN_EDEVICE;
    g_dev[dev].lds_max = (size_t)v;
    g_dev[dev].ok = 1;
  }
  *out = g_dev[dev];
  return SHEN_OK;
}

inline bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

shen_opts resolve(const shen_opts* o) {
  shen_opts r;
  shen_opts_default(&r);
  if (o) r = *o;
  if (r.refine_max < 0) r.refine_max = 8;
  if (!(r.refine_tol > 0.0)) r.refine_tol = 1e-14;
  return r;
}

int check_opts(const shen_opts& o) {
  if (o.precision != SHEN_FP64 && o.precision != SHEN_FP32_REFINE) return SHEN_EINVAL;
  if (o.quad != SHEN_QUAD_GC && o.quad != SHEN_QUAD_GL) return SHEN_EINVAL;
  if (o.transpose != 0 && o.transpose != 1) return SHEN_EINVAL;
  if (o.variant < 0 || o.variant > 2) return SHEN_EINVAL;
  if (o.info && !aligned(o.info, 4)) return SHEN_EINVAL;
  if (o.iters && !aligned(o.iters, 4)) return SHEN_EINVAL;
  if (o.refine_max > 64) return SHEN_EINVAL;
  if (o.chunk < 0 || o.chunk > 64) return SHEN_EINVAL;
  if (o.work_bytes < 0 || (o.work && !aligned(o.work, 16))) return SHEN_EINVAL;
  return SHEN_OK;
}

// opts.chunk: 0, or a chunk length that a wave configuration of (family, N)
// offers; anything else is refused rather than silently replaced.
int check_chunk(const shen_opts& o, int family, int32_t N) {
  return shen::wave_chunk_ok(family, N, o.chunk) ? SHEN_OK : SHEN_EINVAL;
}

// nsys beyond SHEN_MAX_NSYS is refused before anything is launched
inline bool bad_nsys(int64_t nsys) { return nsys < 0 || nsys > SHEN_MAX_NSYS; }

bool rows_overlap_partially(const void* a, const void* b, int64_t nsys, int32_t N) {
  if (a == b) return false;
  const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
  const uintptr_t len = (uintptr_t)nsys * (uintptr_t)N * 16u;
  return pa < pb + len && pb < pa + len;
}

int check_rows(const void* p) { return (p && aligned(p, 16)) ? SHEN_OK : SHEN_EINVAL; }
int check_coef(const void* p) { return (p && aligned(p, 8)) ? SHEN_OK : SHEN_EINVAL; }

int lds_budget_for(ChainKind kind, int N, const DevInfo& d, size_t* budget) {
  const size_t per = shen::chain_bytes_per_system(kind, N) + 4;
  if (per > d.lds_max) return SHEN_ENOTSUP;
  size_t b = 65536;
  if (b > d.lds_max) b = d.lds_max;
  if (per > b) b = per;  // one system per block, up to the device limit
  *budget = b;
  return SHEN_OK;
}

int run(ChainArgs& a) {
  DevInfo d;
  int rc = device_info(&d);
  if (rc != SHEN_OK) return rc;
  rc = lds_budget_for(a.kind, a.N, d, &a.lds_budget);
  if (rc != SHEN_OK) return rc;
  return shen::launch_chain(a) == hipSuccess ? SHEN_OK : SHEN_ELAUNCH;
}

// The wave path serves plain FP64 forward solves out of place (it parks the LU
// restart states in u); everything else, and sizes it does not cover, goes to
// the chain kernels.
// The wave kernels cover the plain FP64 and the FP32 + refinement solves of
// both families here; the transposed solve reaches them through the adjoint
// (use_adjoint_wave).
bool wave_mode_ok(const shen_opts& o, int family) {
  (void)family;
  return !o.transpose;
}
// The transposed FP64 solve H^T u = f is the adjoint solve without gradients:
// out of place, at N with a wave configuration, it runs on the adjoint wave
// kernels.
bool use_adjoint_wave(const shen_opts& o, int family, int32_t N, const void* f, const void* u) {
  return o.transpose && o.precision == SHEN_FP64 && o.variant != SHEN_VARIANT_CHAIN && f != u &&
         shen::wave_supported(family, N);
}
bool use_wave(const shen_opts& o, int family, int32_t N, const void* f, const void* u) {
  if (o.variant == SHEN_VARIANT_CHAIN) return false;
  if (o.variant == SHEN_VARIANT_WAVE) return true;  // caller insists: unsupported -> ENOTSUP
  return wave_mode_ok(o, family) && f != u && shen::wave_supported(family, N);
}

int run_wave(const shen::WaveArgs& w) {
  DevInfo d;
  const int rc = device_info(&d);
  if (rc != SHEN_OK) return rc;
  return shen::launch_wave(w) == hipSuccess ? SHEN_OK : SHEN_ELAUNCH;
}
// Large N on the wave path (chains across the wavefronts of a work group):
// plain FP64 forward solves out of place, past the one-wavefront sizes.
bool use_multi(const shen_opts& o, int family, int32_t N, const void* f, const void* u) {
  return o.variant != SHEN_VARIANT_CHAIN && !o.transpose && o.precision == SHEN_FP64 && f != u &&
         shen::multi_waves(family, N) > 0;
}
int run_multi(const shen::WaveArgs& w) {
  DevInfo d;
  const int rc = device_info(&d);
  if (rc != SHEN_OK) return rc;
  return shen::launch_multi(w) == hipSuccess ? SHEN_OK : SHEN_ELAUNCH;
}

int32_t max_n_for(ChainKind kind, const DevInfo& d) {
  int32_t lo = 5, hi = 1 << 20;
  while (lo < hi) {  // largest N with one system fitting
    const int32_t mid = lo + (hi - lo + 1) / 2;
    if (shen::chain_bytes_per_system(kind, mid) + 4 <= d.lds_max)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Factor-once mode (mode 1: boundary walk into fac; 2: wave solve from fac).
int factored(int family, int32_t N, int64_t nsys, const double* c0, const double* c1, void* fac, const shen_c128* f, shen_c128* u,
             const shen_opts* opts, int mode) {
  const shen_opts o = resolve(opts);
  int rc = check_opts(o);
  if (rc) return rc;
  if (N < (family == SHEN_HELMHOLTZ ? 3 : 5) || bad_nsys(nsys) || check_chunk(o, family, N)) return SHEN_EINVAL;
  if (nsys == 0) return SHEN_OK;
  if (!fac || !aligned(fac, 16) || check_coef(c0) || (family == SHEN_BIHARMONIC && check_coef(c1))) return SHEN_EINVAL;
  const int64_t slot = shen::wave_state_slot(family, N, o.chunk);
  if (mode == 2) {
    if (check_rows(f) || check_rows(u)) return SHEN_EINVAL;
    if (rows_overlap_partially(f, u, nsys, N)) return SHEN_EINVAL;
    // the state slots must not share memory with the solution rows
    const uintptr_t pa = (uintptr_t)fac, pb = (uintptr_t)u;
    const uintptr_t la = (uintptr_t)nsys * (uintptr_t)(slot > 0 ? slot : 1) * 16u, lb = (uintptr_t)nsys * (uintptr_t)N * 16u;
    if (pa < pb + lb && pb < pa + la) return SHEN_EINVAL;
  }
  if (o.precision != SHEN_FP64 || o.transpose || o.variant == SHEN_VARIANT_CHAIN) return SHEN_ENOTSUP;
  if (slot == 0) return SHEN_ENOTSUP;
  shen::WaveArgs w;
  w.family = family;
  w.N = N;
  w.nsys = nsys;
  w.c0 = c0;
  w.c1 = c1;
  w.f = f;
  w.u = u;
  w.info = mode == 2 ? o.info : nullptr;
  w.gl = o.quad == SHEN_QUAD_GL;
  w.chunk = o.chunk;
  w.stream = o.stream;
  w.fac = fac;
  w.fac_mode = mode;
  return shen::multi_waves(family, N) > 0 ? run_multi(w) : run_wave(w);
}

// In-place FP64 solves on the wave kernels through the caller's workspace
// (opts.work): the boundary walk parks its restart states there instead of in
// u (a factor call), then the factored solve runs in place.
bool use_inplace_wave(const shen_opts& o, int family, int32_t N, const void* f, const void* u) {
  return f == u && o.work && o.variant != SHEN_VARIANT_CHAIN && !o.transpose && o.precision == SHEN_FP64 &&
         (shen::wave_supported(family, N) || shen::multi_waves(family, N) > 0);
}
int inplace_wave(int family, int32_t N, int64_t nsys, const double* c0, const double* c1, const shen_c128* f, shen_c128* u,
                 const shen_opts& o) {
  const int64_t slot = shen::wave_state_slot(family, N, o.chunk);
  if (slot <= 0) return SHEN_ENOTSUP;
  const int64_t need = nsys * slot * 16;
  if (o.work_bytes < need) return SHEN_EINVAL;
  const uintptr_t pw = (uintptr_t)o.work, pu = (uintptr_t)u, lu = (uintptr_t)nsys * (uintptr_t)N * 16u;
  if (pw < pu + lu && pu < pw + (uintptr_t)need) return SHEN_EINVAL;  // workspace inside the rows
  shen_opts of = o;
  of.info = nullptr;
  of.work = nullptr;
  of.work_bytes = 0;
  int rc = factored(family, N, nsys, c0, c1, o.work, nullptr, nullptr, &of, 1);
  if (rc != SHEN_OK) return rc;
  shen_opts os = o;
  os.work = nullptr;
  os.work_bytes = 0;
  return factored(family, N, nsys, c0, c1, o.work, f, u, &os, 2);
}

// Adjoint with the restart states of a factor call (no walk; lambda may alias gbar).
int adjoint_factored(int family, int32_t N, int64_t nsys, const double* c0, const double* c1, const void* fac,
                     const shen_c128* u, const shen_c128* gbar, shen_c128* lambda, double* g0, double* g1,
                     const shen_opts* opts) {
  const shen_opts o = resolve(opts);
  int rc = check_opts(o);
  if (rc) return rc;
  if (N < (family == SHEN_HELMHOLTZ ? 3 : 5) || bad_nsys(nsys) || check_chunk(o, family, N)) return SHEN_EINVAL;
  if (nsys == 0) return SHEN_OK;
  if (!fac || !aligned(fac, 16) || check_rows(gbar) || check_rows(lambda) || check_coef(c0) ||
      (family == SHEN_BIHARMONIC && check_coef(c1)))
    return SHEN_EINVAL;
  const bool grads = g0 || g1;
  if (grads && check_rows(u)) return SHEN_EINVAL;
  if ((g0 && !aligned(g0, 8)) || (g1 && !aligned(g1, 8))) return SHEN_EINVAL;
  if (rows_overlap_partially(gbar, lambda, nsys, N)) return SHEN_EINVAL;
  if (u && grads && (u == lambda || rows_overlap_partially(u, lambda, nsys, N))) return SHEN_EINVAL;
  const int64_t slot = shen::wave_state_slot(family, N, o.chunk);
  {
    const uintptr_t pa = (uintptr_t)fac, pb = (uintptr_t)lambda;
    const uintptr_t la = (uintptr_t)nsys * (uintptr_t)(slot > 0 ? slot : 1) * 16u, lb = (uintptr_t)nsys * (uintptr_t)N * 16u;
    if (pa < pb + lb && pb < pa + la) return SHEN_EINVAL;
  }
  // (no adjoint past the one-wavefront sizes on the wave kernels)
  if (o.variant == SHEN_VARIANT_CHAIN || slot == 0 || shen::multi_waves(family, N) > 0) return SHEN_ENOTSUP;
  shen::WaveArgs w;
  w.family = family;
  w.N = N;
  w.nsys = nsys;
  w.c0 = c0;
  w.c1 = c1;
  w.f = gbar;
  w.u = lambda;
  w.info = o.info;
  w.gl = o.quad == SHEN_QUAD_GL;
  w.chunk = o.chunk;
  w.adjoint = 1;
  w.ufwd = grads ? u : nullptr;
  w.g0 = g0;
  w.g1 = g1;
  w.stream = o.stream;
  w.fac = const_cast<void*>(fac);
  w.fac_mode = 2;
  return run_wave(w);
}

// Mass-matrix solves u = B^{-1} f (wave kernels only; u may alias f).
int mass_solve(int family, int32_t N, int64_t nsys, const shen_c128* f, shen_c128* u, const shen_opts* opts, int deriv = 0) {
  const shen_opts o = resolve(opts);
  int rc = check_opts(o);
  if (rc) return rc;
  if (N < (family == SHEN_HELMHOLTZ && !deriv ? 3 : 5) || bad_nsys(nsys)) return SHEN_EINVAL;
  if (o.precision != SHEN_FP64) return SHEN_ENOTSUP;
  if (o.variant == SHEN_VARIANT_CHAIN || !shen::mass_wave_supported(N)) return SHEN_ENOTSUP;
  if (nsys == 0) return SHEN_OK;
  if (check_rows(f) || check_rows(u)) return SHEN_EINVAL;
  if (rows_overlap_partially(f, u, nsys, N)) return SHEN_EINVAL;
  DevInfo d;
  rc = device_info(&d);
  if (rc != SHEN_OK) return rc;
  shen::WaveArgs w;
  w.family = family;
  w.N = N;
  w.nsys = nsys;
  w.f = f;
  w.u = u;
  w.gl = o.quad == SHEN_QUAD_GL;
  w.stream = o.stream;
  w.deriv = deriv;
  return shen::launch_mass_wave(w) == hipSuccess ? SHEN_OK : SHEN_ELAUNCH;
}

}  // namespace

extern "C" {

void shen_opts_default(shen_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->precision = SHEN_FP64;
  o->quad = SHEN_QUAD_GC;
  o->refine_max = 8;
  o->refine_tol = 1e-14;
}

int shen_abi_version(void) { return SHENHIP_ABI_VERSION; }

const char* shen_status_string(int code) {
  switch (code) {
    case SHEN_OK: return "ok";
    case SHEN_EINVAL: return "invalid argument";
    case SHEN_ELAUNCH: return "kernel launch failed";
    case SHEN_ENOTSUP: return "size not supported by this kernel on this device";
    case SHEN_EDEVICE: return "no usable HIP device";
    case SHEN_ESCRATCH: return "the call needs more scratch than the library's static buffer holds";
    default: return "unknown status";
  }
}

int shen_wave_config(int32_t family, int32_t N, int32_t chunk, int32_t* C, int32_t* G) {
  if (family != SHEN_HELMHOLTZ && family != SHEN_BIHARMONIC) return SHEN_EINVAL;
  if (N < (family == SHEN_HELMHOLTZ ? 3 : 5) || chunk < 0 || chunk > 64) return SHEN_EINVAL;
  if (!shen::wave_supported(family, N)) return SHEN_ENOTSUP;
  if (!shen::wave_chunk_ok(family, N, chunk)) return SHEN_EINVAL;
  const shen::WaveCfg c = shen::pick_cfg((N + 1) / 2, family, N, chunk);
  if (C) *C = c.C;
  if (G) *G = c.G;
  return SHEN_OK;
}

int32_t shen_max_n(int32_t family, int32_t precision) {
  DevInfo d;
  if (device_info(&d) != SHEN_OK) return SHEN_EDEVICE;
  ChainKind k;
  if (family == SHEN_HELMHOLTZ)
    k = precision == SHEN_FP32_REFINE ? ChainKind::HelmMixed : ChainKind::HelmSolve;
  else if (family == SHEN_BIHARMONIC)
    k = precision == SHEN_FP32_REFINE ? ChainKind::BihMixed : ChainKind::BihSolve;
  else
    return SHEN_EINVAL;
  int32_t nmax = max_n_for(k, d);
  if (precision == SHEN_FP64) {  // the large-N wave solves (out of place)
    int32_t top = nmax;
    for (int32_t N = 1025; N <= 8192; ++N)
      if (shen::multi_waves(family, N) > 0) top = N;
    nmax = top > nmax ? top : nmax;
  }
  return nmax;
}

int helmholtz_solve(int32_t N, int64_t nsys, const double* alpha, const shen_c128* f, shen_c128* u, const shen_opts* opts) {
  const shen_opts o = resolve(opts);
  int rc = check_opts(o);
  if (rc) return rc;
  if (N < 3 || bad_nsys(nsys) || check_chunk(o, SHEN_HELMHOLTZ, N)) return SHEN_EINVAL;
  if (nsys == 0) return SHEN_OK;
  if (check_rows(f) || check_rows(u) || check_coef(alpha)) return SHEN_EINVAL;
  if (rows_overlap_partially(f, u, nsys, N)) return SHEN_EINVAL;
  if (o.transpose && o.precision != SHEN_FP64) return SHEN_ENOTSUP;
  if (use_adjoint_wave(o, 0, N, f, u)) return helmholtz_adjoint(N, nsys, alpha, nullptr, f, u, nullptr, opts);
  if (use_inplace_wave(o, 0, N, f, u)) return inplace_wave(SHEN_HELMHOLTZ, N, nsys, alpha, nullptr, f, u, o);
  if (use_multi(o, 0, N, f, u)) {
    shen::WaveArgs w;
    w.family = 0;
    w.N = N;
    w.nsys = nsys;
    w.c0 = alpha;
    w.f = f;
    w.u = u;
    w.info = o.info;
    w.gl = o.quad == SHEN_QUAD_GL;
    w.stream = o.stream;
    return run_multi(w);
  }
  if (use_wave(o, 0, N, f, u)) {
    if (!wave_mode_ok(o, 0) || !shen::wave_supported(0, N) || f == (const void*)u) return SHEN_ENOTSUP;
    shen::WaveArgs w;
    w.family = 0;
    w.mixed = o.precision == SHEN_FP32_REFINE;
    w.it_max = o.refine_max;
    w.tol = o.refine_tol;
    w.N = N;
    w.nsys = nsys;
    w.c0 = alpha;
    w.f = f;
    w.u = u;
    w.info = o.info;
    w.iters = w.mixed ? o.iters : nullptr;
    w.gl = o.quad == SHEN_QUAD_GL;
    w.chunk = o.chunk;
    w.stream = o.stream;
    return run_wave(w);
  }
  ChainArgs a;
  a.iters = o.precision == SHEN_FP32_REFINE ? o.iters : nullptr;
  a.kind = o.transpose ? ChainKind::HelmAdjoint : (o.precision == SHEN_FP32_REFINE ? ChainKind::HelmMixed : ChainKind::HelmSolve);
  a.N = N;
  a.nsys = nsys;
  a.c0 = alpha;
  a.f = f;
  a.u = u;
  a.info = o.info;
  a.gl = o.quad == SHEN_QUAD_GL;
  a.it_max = o.refine_max;
  a.tol = o.refine_tol;
  a.stream = o.stream;
  return run(a);
}

int biharmonic_solve(int32_t N, int64_t nsys, const double* ca, const double* cb, const shen_c128* f, shen_c128* u,
                     const shen_opts* opts) {
  const shen_opts o = resolve(opts);
  int rc = check_opts(o);
  if (rc) return rc;
  if (N < 5 || bad_nsys(nsys) || check_chunk(o, SHEN_BIHARMONIC, N)) return SHEN_EINVAL;
  if (nsys == 0) return SHEN_OK;
  if (check_rows(f) || check_rows(u) || check_coef(ca) || check_coef(cb)) return SHEN_EINVAL;
  if (rows_overlap_partially(f, u, nsys, N)) return SHEN_EINVAL;
  if (o.transpose && o.precision != SHEN_FP64) return SHEN_ENOTSUP;
  if (use_adjoint_wave(o, 1, N, f, u)) return biharmonic_adjoint(N, nsys, ca, cb, nullptr, f, u, nullptr, nullptr, opts);
  if (use_inplace_wave(o, 1, N, f, u)) return inplace_wave(SHEN_BIHARMONIC, N, nsys, ca, cb, f, u, o);
  if (use_multi(o, 1, N, f, u)) {
    shen::WaveArgs w;
    w.family = 1;
    w.N = N;
    w.nsys = nsys;
    w.c0 = ca;
    w.c1 = cb;
    w.f = f;
    w.u = u;
    w.info = o.info;
    w.gl = o.quad == SHEN_QUAD_GL;
    w.stream = o.stream;
    return run_multi(w);
  }
  if (use_wave(o, 1, N, f, u)) {
    if (!wave_mode_ok(o, 1) || !shen::wave_supported(1, N) || f == (const void*)u) return SHEN_ENOTSUP;
    shen::WaveArgs w;
    w.family = 1;
    w.mixed = o.precision == SHEN_FP32_REFINE;
    w.it_max = o.refine_max;
    w.tol = o.refine_tol;
    w.N = N;
    w.nsys = nsys;
    w.c0 = ca;
    w.c1 = cb;
    w.f = f;
    w.u = u;
    w.info = o.info;
    w.iters = w.mixed ? o.iters : nullptr;
    w.gl = o.quad == SHEN_QUAD_GL;
    w.chunk = o.chunk;
    w.stream = o.stream;
    return run_wave(w);
  }
  ChainArgs a;
  a.iters = o.precision == SHEN_FP32_REFINE ? o.iters : nullptr;
  a.kind = o.transpose ? ChainKind::BihAdjoint : (o.precision == SHEN_FP32_REFINE ? ChainKind::BihMixed : ChainKind::BihSolve);
  a.N = N;
  a.nsys = nsys;
  a.c0 = ca;
  a.c1 = cb;
  a.f = f;
  a.u = u;
  a.info = o.info;
  a.gl = o.quad == SHEN_QUAD_GL;
  a.it_max = o.refine_max;
  a.tol = o.refine_tol;
  a.stream = o.stream;
  return run(a);
}

int helmholtz_adjoint(int32_t N, int64_t nsys, const double* alpha, const shen_c128* u, const shen_c128* gbar, shen_c128* lambda,
                      double* grad_alpha, const shen_opts* opts) {
  const shen_opts o = resolve(opts);
  int rc = check_opts(o);
  if (rc) return rc;
  if (N < 3 || bad_nsys(nsys) || check_chunk(o, SHEN_HELMHOLTZ, N)) return SHEN_EINVAL;
  if (nsys == 0) return SHEN_OK;
  if (check_rows(gbar) || check_rows(lambda) || check_coef(alpha)) return SHEN_EINVAL;
  if (grad_alpha && (check_rows(u) || !aligned(grad_alpha, 8))) return SHEN_EINVAL;
  if (rows_overlap_partially(gbar, lambda, nsys, N)) return SHEN_EINVAL;
  if (u && (u == lambda || rows_overlap_partially(u, lambda, nsys, N))) return SHEN_EINVAL;
  if (o.variant != SHEN_VARIANT_CHAIN && (const void*)gbar != (const void*)lambda && shen::wave_supported(0, N)) {
    shen::WaveArgs w;
    w.family = 0;
    w.N = N;
    w.nsys = nsys;
    w.c0 = alpha;
    w.f = gbar;
    w.u = lambda;
    w.info = o.info;
    w.gl = o.quad == SHEN_QUAD_GL;
    w.chunk = o.chunk;
    w.adjoint = 1;
    w.ufwd = grad_alpha ? u : nullptr;
    w.g0 = grad_alpha;
    w.stream = o.stream;
    return run_wave(w);
  }
  if (o.variant == SHEN_VARIANT_WAVE) return SHEN_ENOTSUP;
  ChainArgs a;
  a.kind = ChainKind::HelmAdjoint;
  a.N = N;
  a.nsys = nsys;
  a.c0 = alpha;
  a.f = gbar;
  a.u = lambda;
  a.ufwd = grad_alpha ? u : nullptr;
  a.g0 = grad_alpha;
  a.info = o.info;
  a.gl = o.quad == SHEN_QUAD_GL;
  a.stream = o.stream;
  return run(a);
}

int biharmonic_adjoint(int32_t N, int64_t nsys, const double* ca, const double* cb, const shen_c128* u, const shen_c128* gbar,
                       shen_c128* lambda, double* grad_a, double* grad_b, const shen_opts* opts) {
  const shen_opts o = resolve(opts);
  int rc = check_opts(o);
  if (rc) return rc;
  if (N < 5 || bad_nsys(nsys) || check_chunk(o, SHEN_BIHARMONIC, N)) return SHEN_EINVAL;
  if (nsys == 0) return SHEN_OK;
  if (check_rows(gbar) || check_rows(lambda) || check_coef(ca) || check_coef(cb)) return SHEN_EINVAL;
  const bool grads = grad_a || grad_b;
  if (grads && check_rows(u)) return SHEN_EINVAL;
  if ((grad_a && !aligned(grad_a, 8)) || (grad_b && !aligned(grad_b, 8))) return SHEN_EINVAL;
  if (rows_overlap_partially(gbar, lambda, nsys, N)) return SHEN_EINVAL;
  if (u && (u == lambda || rows_overlap_partially(u, lambda, nsys, N))) return SHEN_EINVAL;
  if (o.variant != SHEN_VARIANT_CHAIN && (const void*)gbar != (const void*)lambda && shen::wave_supported(1, N)) {
    shen::WaveArgs w;
    w.family = 1;
    w.N = N;
    w.nsys = nsys;
    w.c0 = ca;
    w.c1 = cb;
    w.f = gbar;
    w.u = lambda;
    w.info = o.info;
    w.gl = o.quad == SHEN_QUAD_GL;
    w.chunk = o.chunk;
    w.adjoint = 1;
    w.ufwd = grads ? u : nullptr;
    w.g0 = grad_a;
    w.g1 = grad_b;
    w.stream = o.stream;
    return run_wave(w);
  }
  if (o.variant == SHEN_VARIANT_WAVE) return SHEN_ENOTSUP;
  ChainArgs a;
  a.kind = ChainKind::BihAdjoint;
  a.N = N;
  a.nsys = nsys;
  a.c0 = ca;
  a.c1 = cb;
  a.f = gbar;
  a.u = lambda;
  a.ufwd = grads ? u : nullptr;
  a.g0 = grad_a;
  a.g1 = grad_b;
  a.info = o.info;
  a.gl = o.quad == SHEN_QUAD_GL;
  a.stream = o.stream;
  return run(a);
}

int helmholtz_adjoint_factored(int32_t N, int64_t nsys, const double* alpha, const void* fac, const shen_c128* u,
                               const shen_c128* gbar, shen_c128* lambda, double* grad_alpha, const shen_opts* opts) {
  return adjoint_factored(SHEN_HELMHOLTZ, N, nsys, alpha, nullptr, fac, u, gbar, lambda, grad_alpha, nullptr, opts);
}
int biharmonic_adjoint_factored(int32_t N, int64_t nsys, const double* a, const double* b, const void* fac, const shen_c128* u,
                                const shen_c128* gbar, shen_c128* lambda, double* grad_a, double* grad_b,
                                const shen_opts* opts) {
  return adjoint_factored(SHEN_BIHARMONIC, N, nsys, a, b, fac, u, gbar, lambda, grad_a, grad_b, opts);
}

int64_t shen_factor_bytes(int32_t family, int32_t N, const shen_opts* opts) {
  const shen_opts o = resolve(opts);
  if (check_opts(o)) return SHEN_EINVAL;
  if (family != SHEN_HELMHOLTZ && family != SHEN_BIHARMONIC) return SHEN_EINVAL;
  if (N < (family == SHEN_HELMHOLTZ ? 3 : 5) || check_chunk(o, family, N)) return SHEN_EINVAL;
  const int64_t slot = shen::wave_state_slot(family, N, o.chunk);
  return slot > 0 ? slot * 16 : SHEN_ENOTSUP;
}

int helmholtz_factor(int32_t N, int64_t nsys, const double* alpha, void* fac, const shen_opts* opts) {
  return factored(SHEN_HELMHOLTZ, N, nsys, alpha, nullptr, fac, nullptr, nullptr, opts, 1);
}
int biharmonic_factor(int32_t N, int64_t nsys, const double* a, const double* b, void* fac, const shen_opts* opts) {
  return factored(SHEN_BIHARMONIC, N, nsys, a, b, fac, nullptr, nullptr, opts, 1);
}
int helmholtz_solve_factored(int32_t N, int64_t nsys, const double* alpha, const void* fac, const shen_c128* f, shen_c128* u,
                             const shen_opts* opts) {
  return factored(SHEN_HELMHOLTZ, N, nsys, alpha, nullptr, const_cast<void*>(fac), f, u, opts, 2);
}
int biharmonic_solve_factored(int32_t N, int64_t nsys, const double* a, const double* b, const void* fac, const shen_c128* f,
                              shen_c128* u, const shen_opts* opts) {
  return factored(SHEN_BIHARMONIC, N, nsys, a, b, const_cast<void*>(fac), f, u, opts, 2);
}

int helmholtz_matvec(int32_t N, int64_t nsys, const double* alpha, const shen_c128* u, shen_c128* Hu, const shen_opts* opts) {
  const shen_opts o = resolve(opts);
  int rc = check_opts(o);
  if (rc) return rc;
  if (N < 3 || bad_nsys(nsys)) return SHEN_EINVAL;
  if (nsys == 0) return SHEN_OK;
  if (check_rows(u) || check_rows(Hu) || check_coef(alpha)) return SHEN_EINVAL;
  if (u == Hu || rows_overlap_partially(u, Hu, nsys, N)) return SHEN_EINVAL;
  if (!o.transpose && o.variant != SHEN_VARIANT_CHAIN && shen::matvec_wave_supported(0, N)) {
    shen::WaveArgs w;
    w.family = 0;
    w.N = N;
    w.nsys = nsys;
    w.c0 = alpha;
    w.f = u;
    w.u = Hu;
    w.gl = o.quad == SHEN_QUAD_GL;
    w.stream = o.stream;
    DevInfo d;
    const int rc2 = device_info(&d);
    if (rc2 != SHEN_OK) return rc2;
    return shen::launch_matvec_wave(w) == hipSuccess ? SHEN_OK : SHEN_ELAUNCH;
  }
  ChainArgs a;
  a.kind = ChainKind::HelmMatvec;
  a.N = N;
  a.nsys = nsys;
  a.c0 = alpha;
  a.f = u;
  a.u = Hu;
  a.gl = o.quad == SHEN_QUAD_GL;
  a.trans = o.transpose;
  a.stream = o.stream;
  return run(a);
}

int biharmonic_matvec(int32_t N, int64_t nsys, const double* ca, const double* cb, const shen_c128* u, shen_c128* Hu,
                      const shen_opts* opts) {
  const shen_opts o = resolve(opts);
  int rc = check_opts(o);
  if (rc) return rc;
  if (N < 5 || bad_nsys(nsys)) return SHEN_EINVAL;
  if (nsys == 0) return SHEN_OK;
  if (check_rows(u) || check_rows(Hu) || check_coef(ca) || check_coef(cb)) return SHEN_EINVAL;
  if (u == Hu || rows_overlap_partially(u, Hu, nsys, N)) return SHEN_EINVAL;
  if (!o.transpose && o.variant != SHEN_VARIANT_CHAIN && shen::matvec_wave_supported(1, N)) {
    shen::WaveArgs w;
    w.family = 1;
    w.N = N;
    w.nsys = nsys;
    w.c0 = ca;
    w.c1 = cb;
    w.f = u;
    w.u = Hu;
    w.gl = o.quad == SHEN_QUAD_GL;
    w.stream = o.stream;
    DevInfo d;
    const int rc2 = device_info(&d);
    if (rc2 != SHEN_OK) return rc2;
    return shen::launch_matvec_wave(w) == hipSuccess ? SHEN_OK : SHEN_ELAUNCH;
  }
  ChainArgs a;
  a.kind = ChainKind::BihMatvec;
  a.N = N;
  a.nsys = nsys;
  a.c0 = ca;
  a.c1 = cb;
  a.f = u;
  a.u = Hu;
  a.gl = o.quad == SHEN_QUAD_GL;
  a.trans = o.transpose;
  a.stream = o.stream;
  return run(a);
}

// Crank-Nicolson right-hand sides (Sec. 3, eqs. gfin and ufin) on the matvec
// kernels: the coefficients the step maps K2 and 2/(nu dt) to are formed in
// the kernels, the product is negated and sigma S(h) added on the way out.
static int rhs_assemble(int family, int32_t N, int64_t nsys, const double* K2, double nu, double dt, const shen_c128* uhat,
                        const shen_c128* sh, shen_c128* rhs, const shen_opts* opts) {
  const shen_opts o = resolve(opts);
  int rc = check_opts(o);
  if (rc) return rc;
  if (o.transpose) return SHEN_EINVAL;
  if (N < (family == SHEN_HELMHOLTZ ? 3 : 5) || bad_nsys(nsys)) return SHEN_EINVAL;
  if (!(nu > 0.0) || !(dt > 0.0) || !std::isfinite(2.0 / (nu * dt)) || !std::isfinite(2.0 / nu)) return SHEN_EINVAL;
  if (nsys == 0) return SHEN_OK;
  if (check_rows(uhat) || check_rows(rhs) || check_coef(K2) || (sh && check_rows(sh))) return SHEN_EINVAL;
  if ((const void*)uhat == (const void*)rhs || rows_overlap_partially(uhat, rhs, nsys, N)) return SHEN_EINVAL;
  if (sh && (const void*)sh != (const void*)rhs && rows_overlap_partially(sh, rhs, nsys, N)) return SHEN_EINVAL;
  const double inv = 2.0 / (nu * dt);
  const double sigma = (family == SHEN_HELMHOLTZ ? 2.0 : -2.0) / nu;
  if (o.variant != SHEN_VARIANT_CHAIN && shen::matvec_wave_supported(family, N)) {
    shen::WaveArgs w;
    w.family = family;
    w.N = N;
    w.nsys = nsys;
    w.c0 = K2;
    w.c1 = K2;
    w.f = uhat;
    w.u = rhs;
    w.gl = o.quad == SHEN_QUAD_GL;
    w.stream = o.stream;
    w.rhs = 1;
    w.inv = inv;
    w.sigma = sigma;
    w.sh = sh;
    DevInfo d;
    const int rc2 = device_info(&d);
    if (rc2 != SHEN_OK) return rc2;
    return shen::launch_matvec_wave(w) == hipSuccess ? SHEN_OK : SHEN_ELAUNCH;
  }
  ChainArgs a;
  a.kind = family == SHEN_HELMHOLTZ ? ChainKind::HelmMatvec : ChainKind::BihMatvec;
  a.N = N;
  a.nsys = nsys;
  a.c0 = K2;
  a.c1 = K2;
  a.f = uhat;
  a.u = rhs;
  a.gl = o.quad == SHEN_QUAD_GL;
  a.trans = 0;
  a.stream = o.stream;
  a.rhs = 1;
  a.inv = inv;
  a.sigma = sigma;
  a.sh = sh;
  return run(a);
}

int helmholtz_rhs(int32_t N, int64_t nsys, const double* K2, double nu, double dt, const shen_c128* ghat,
                  const shen_c128* sh, shen_c128* rhs, const shen_opts* opts) {
  return rhs_assemble(SHEN_HELMHOLTZ, N, nsys, K2, nu, dt, ghat, sh, rhs, opts);
}
int biharmonic_rhs(int32_t N, int64_t nsys, const double* K2, double nu, double dt, const shen_c128* uhat,
                   const shen_c128* sh, shen_c128* rhs, const shen_opts* opts) {
  return rhs_assemble(SHEN_BIHARMONIC, N, nsys, K2, nu, dt, uhat, sh, rhs, opts);
}

// Shen transforms: validation, then the transform kernel (and, for the
// forward transform of the Dirichlet and biharmonic spaces, the mass solve
// in place on the scalar products).
static int transform_args(int32_t N, int64_t nsys, int32_t space, const void* in, const void* out, const shen_opts& o,
                          int dir, int forward_solve) {
  if (check_opts(o)) return SHEN_EINVAL;
  if (space != SHEN_SPACE_CHEBYSHEV && space != SHEN_SPACE_DIRICHLET && space != SHEN_SPACE_BIHARMONIC) return SHEN_EINVAL;
  const int nmin = space == SHEN_SPACE_CHEBYSHEV ? 1 : (space == SHEN_SPACE_DIRICHLET ? 3 : 5);
  if (N < nmin || bad_nsys(nsys) || o.transpose) return SHEN_EINVAL;
  if (N > 2048) return SHEN_ENOTSUP;
  if (dir == 0 && forward_solve && space != SHEN_SPACE_CHEBYSHEV && !shen::mass_wave_supported(N)) return SHEN_ENOTSUP;
  if (nsys == 0) return SHEN_OK;
  if (check_rows(in) || check_rows(out)) return SHEN_EINVAL;
  if (in == out || rows_overlap_partially(in, out, nsys, N)) return SHEN_EINVAL;
  const int gl = o.quad == SHEN_QUAD_GL;
  if (!shen::transform_fft_ok(N, gl) && shen::transform_direct_lds(N, gl, nullptr) > 160 * 1024) return SHEN_ENOTSUP;
  return SHEN_OK + 1;  // valid, work to do
}

int shen_scalar_product(int32_t N, int64_t nsys, int32_t space, const shen_c128* u, shen_c128* s, const shen_opts* opts) {
  const shen_opts o = resolve(opts);
  const int rc = transform_args(N, nsys, space, u, s, o, 0, 0);
  if (rc <= 0) return rc;
  DevInfo d;
  const int rc2 = device_info(&d);
  if (rc2 != SHEN_OK) return rc2;
  return shen::launch_transform(N, nsys, space, 0, 0, o.quad == SHEN_QUAD_GL, u, s, o.stream) == hipSuccess ? SHEN_OK
                                                                                                             : SHEN_ELAUNCH;
}

int shen_forward_transform(int32_t N, int64_t nsys, int32_t space, const shen_c128* u, shen_c128* uhat,
                           const shen_opts* opts) {
  const shen_opts o = resolve(opts);
  const int rc = transform_args(N, nsys, space, u, uhat, o, 0, 1);
  if (rc <= 0) return rc;
  DevInfo d;
  const int rc2 = device_info(&d);
  if (rc2 != SHEN_OK) return rc2;
  const int chebyshev = space == SHEN_SPACE_CHEBYSHEV;
  // the FFT kernel solves the Dirichlet mass matrix itself (one pass)
  const int fused = space == SHEN_SPACE_DIRICHLET && shen::transform_fused_mass_ok(N, o.quad == SHEN_QUAD_GL);
  if (shen::launch_transform(N, nsys, space, 0, chebyshev || fused, o.quad == SHEN_QUAD_GL, u, uhat, o.stream) != hipSuccess)
    return SHEN_ELAUNCH;
  if (chebyshev || fused) return SHEN_OK;
  shen_opts om = o;
  om.variant = 0;
  return mass_solve(space == SHEN_SPACE_DIRICHLET ? SHEN_HELMHOLTZ : SHEN_BIHARMONIC, N, nsys, uhat, uhat, &om);
}

int shen_backward_transform(int32_t N, int64_t nsys, int32_t space, const shen_c128* uhat, shen_c128* u,
                            const shen_opts* opts) {
  const shen_opts o = resolve(opts);
  const int rc = transform_args(N, nsys, space, uhat, u, o, 1, 0);
  if (rc <= 0) return rc;
  DevInfo d;
  const int rc2 = device_info(&d);
  if (rc2 != SHEN_OK) return rc2;
  return shen::launch_transform(N, nsys, space, 1, 0, o.quad == SHEN_QUAD_GL, uhat, u, o.stream) == hipSuccess
             ? SHEN_OK
             : SHEN_ELAUNCH;
}

int dirichlet_mass_solve(int32_t N, int64_t nsys, const shen_c128* f, shen_c128* u, const shen_opts* opts) {
  return mass_solve(SHEN_HELMHOLTZ, N, nsys, f, u, opts);
}
int biharmonic_mass_solve(int32_t N, int64_t nsys, const shen_c128* f, shen_c128* u, const shen_opts* opts) {
  return mass_solve(SHEN_BIHARMONIC, N, nsys, f, u, opts);
}
int dirichlet_derivative_solve(int32_t N, int64_t nsys, const shen_c128* uhat, shen_c128* fhat, const shen_opts* opts) {
  return mass_solve(SHEN_HELMHOLTZ, N, nsys, uhat, fhat, opts, 1);
}

// Checks one batched descriptor (shared by the plan and the solves, which
// re-read the host descriptors at every call).
static int check_desc(const shen_problem& d) {
  if (d.family != SHEN_HELMHOLTZ && d.family != SHEN_BIHARMONIC) return SHEN_EINVAL;
  if (bad_nsys(d.nsys) || d.N < (d.family == SHEN_HELMHOLTZ ? 3 : 5)) return SHEN_EINVAL;
  if (d.nsys > 0) {
    if (check_rows(d.f) || check_rows(d.u) || check_coef(d.c0)) return SHEN_EINVAL;
    if (d.family == SHEN_BIHARMONIC && check_coef(d.c1)) return SHEN_EINVAL;
    if (d.info && !aligned(d.info, 4)) return SHEN_EINVAL;
    if ((const void*)d.f == (const void*)d.u || rows_overlap_partially(d.f, d.u, d.nsys, d.N)) return SHEN_EINVAL;
  }
  if (shen::multi_waves(d.family, d.N) > 0) {  // large N: no chunk knob
    if (d.chunk != 0) return SHEN_EINVAL;
  } else {
    if (!shen::wave_supported(d.family, d.N)) return SHEN_ENOTSUP;
    if (d.chunk < 0 || d.chunk > 64 || !shen::wave_chunk_ok(d.family, d.N, d.chunk)) return SHEN_EINVAL;
  }
  if (d.sys_per_tile < 0 || d.sys_per_tile > 1 << 20) return SHEN_EINVAL;
  return SHEN_OK;
}

int64_t shen_batched_plan(shen_problem* desc, int32_t ndesc, const shen_opts* opts) {
  const shen_opts o = resolve(opts);
  if (check_opts(o)) return SHEN_EINVAL;
  if (!desc || ndesc <= 0) return SHEN_EINVAL;
  int64_t total = 0;
  for (int32_t i = 0; i < ndesc; ++i) {
    shen_problem& d = desc[i];
    if (d.sys_per_tile == 0) d.sys_per_tile = 32;
    const int rc = check_desc(d);
    if (rc) return rc;
    d.tile_begin = total;
    total += (d.nsys + d.sys_per_tile - 1) / d.sys_per_tile;
  }
  // best effort: where this fails (no device here), batched_solve tries again
  (void)shen::batched_fork_prepare();
  return total;
}

int64_t shen_batched_work_bytes(int32_t ndesc) {
  if (ndesc < 0) return SHEN_EINVAL;
  const int64_t bytes = 8 * (int64_t)shen::batched_counters(ndesc);
  return bytes < 256 ? 256 : (bytes + 255) / 256 * 256;
}

static int batched_common(const shen_problem* desc, int32_t ndesc, const shen_opts& o) {
  int rc = check_opts(o);
  if (rc) return rc;
  if (!desc || !aligned(desc, 8) || ndesc <= 0) return SHEN_EINVAL;
  for (int32_t i = 0; i < ndesc; ++i) {
    if (desc[i].sys_per_tile <= 0) return SHEN_EINVAL;  // not planned
    rc = check_desc(desc[i]);
    if (rc) return rc;
  }
  DevInfo d;
  return device_info(&d);
}

int batched_solve(const shen_problem* desc, int32_t ndesc, void* work, const shen_opts* opts) {
  const shen_opts o = resolve(opts);
  if (!work || !aligned(work, 8)) return SHEN_EINVAL;
  const int rc = batched_common(desc, ndesc, o);
  if (rc) return rc;
  return shen::launch_batched(desc, ndesc, work, o.quad == SHEN_QUAD_GL, o.stream, true) == hipSuccess ? SHEN_OK
                                                                                                        : SHEN_ELAUNCH;
}

int64_t shen_batched_static_bytes(void) { return (int64_t)shen::kBatchedStaticWords * 8; }

int batched_solve_static(const shen_problem* desc, int32_t ndesc, const shen_opts* opts) {
  const shen_opts o = resolve(opts);
  if (check_opts(o)) return SHEN_EINVAL;
  if (!desc || !aligned(desc, 8) || ndesc <= 0) return SHEN_EINVAL;
  const int64_t need = shen_batched_work_bytes(ndesc);
  if (need < 0) return SHEN_EINVAL;
  if (need > shen_batched_static_bytes()) return SHEN_ESCRATCH;
  const int rc = batched_common(desc, ndesc, o);
  if (rc) return rc;
  void* work = nullptr;
  if (shen::batched_static_scratch(&work) != hipSuccess || work == nullptr) return SHEN_EDEVICE;
  // in order on the caller's stream: no side streams or events to create
  return shen::launch_batched(desc, ndesc, work, o.quad == SHEN_QUAD_GL, o.stream, false) == hipSuccess ? SHEN_OK
                                                                                                         : SHEN_ELAUNCH;
}

}  // extern "C"
