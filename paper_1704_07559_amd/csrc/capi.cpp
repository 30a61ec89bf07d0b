// C ABI of the library (include/lbm.h): argument validation, the context, ping-pong of
// the two population buffers and dispatch to the kernel launchers. No exception leaves
// this file; every failure is an lbm_status plus a thread-local message.
#include "../../include/lbm.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "internal.h"
#include "launch.h"

using namespace lbm;

struct lbm_ctx {
  lbm_params p;
  int Q;
  size_t elem;      // bytes per stored population
  size_t pop_bytes; // Q * N * elem
  Geo G;
  ModelF M;
  ViscF V;
  ForceF F;
  void* buf[2];
  int cur;          // buffer holding the current internal state
  float* snu;       // lagged s_nu field (variable viscosity) or nullptr
  float* snu_pair;  // D2Q9 two-step launches with a lagged s_nu: the field between two of them
  double* scratch;  // reduction partials (kReduceBlocks * 8) + result (8)
  long long step;
};

namespace {

thread_local std::string g_last_error;

lbm_status fail(lbm_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

lbm_status hip_fail(hipError_t e, const char* where) {
  g_last_error = std::string(where) + ": " + hipGetErrorString(e);
  return LBM_EHIP;
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

size_t elem_size(int storage) {
  switch (storage) {
    case LBM_F32: return 4;
    case LBM_F16: return 2;
    case LBM_BF16: return 2;
    default: return 0;
  }
}

// Validate the parameters; on success fill Q and N.
lbm_status check_params(const lbm_params* p, int* Q, size_t* N) {
  if (!p) return fail(LBM_EINVAL, "params is NULL");
  if (p->lattice != LBM_D3Q19 && p->lattice != LBM_D3Q15 && p->lattice != LBM_D2Q9)
    return fail(LBM_EINVAL, "lattice must be LBM_D3Q19, LBM_D3Q15 or LBM_D2Q9");
  if (elem_size(p->storage) == 0) return fail(LBM_EINVAL, "storage must be LBM_F32, LBM_F16 or LBM_BF16");
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(LBM_EINVAL, "nx, ny, nz must be >= 1");
  if (p->lattice == LBM_D2Q9 && p->nz != 1) return fail(LBM_EINVAL, "D2Q9 requires nz == 1");
  const size_t n = static_cast<size_t>(p->nx) * p->ny * p->nz;
  if (n >= (size_t(1) << 30)) return fail(LBM_EINVAL, "nx*ny*nz must be below 2^30 nodes");
  // one z-plane of a population buffer (ny rows of Q runs of nx elements) is addressed with
  // 32-bit byte offsets
  if (static_cast<size_t>(p->nx) * p->ny * p->lattice * elem_size(p->storage) >= (size_t(1) << 32))
    return fail(LBM_EINVAL, "nx*ny*Q*element size must be below 2^32 bytes");
  if (!(p->rho0 > 0.0) || !std::isfinite(p->rho0)) return fail(LBM_EINVAL, "rho0 must be positive and finite");
  const int q = p->lattice;
  for (int k = 0; k < q; ++k)
    if (!std::isfinite(p->s[k])) return fail(LBM_EINVAL, "relaxation rates must be finite");
  if (q == 19) {
    const double sn = p->s[9];
    if (p->s[11] != sn || p->s[13] != sn || p->s[14] != sn || p->s[15] != sn)
      return fail(LBM_EINVAL, "D3Q19: the s_nu slots 9, 11, 13, 14, 15 must be equal");
  } else if (q == 15) {
    const double sn = p->s[9];
    if (p->s[10] != sn || p->s[11] != sn || p->s[12] != sn || p->s[13] != sn)
      return fail(LBM_EINVAL, "D3Q15: the s_nu slots 9..13 must be equal");
  } else {
    if (p->s[8] != p->s[7]) return fail(LBM_EINVAL, "D2Q9: the s_nu slots 7 and 8 must be equal");
  }
  const int snu_slot = (q == 9) ? 7 : 9;
  if (!(p->s[snu_slot] > 0.0)) return fail(LBM_EINVAL, "s_nu must be positive");
  if (p->visc_kind < LBM_VISC_CONST || p->visc_kind > LBM_VISC_SMAGORINSKY_IMPLICIT)
    return fail(LBM_EINVAL, "bad visc_kind");
  if (p->visc_kind != LBM_VISC_CONST && p->visc_strain != LBM_STRAIN_YU && p->visc_strain != LBM_STRAIN_CHAI)
    return fail(LBM_EINVAL, "visc_strain must be LBM_STRAIN_YU or LBM_STRAIN_CHAI");
  if ((p->visc_kind == LBM_VISC_SMAGORINSKY || p->visc_kind == LBM_VISC_SMAGORINSKY_IMPLICIT) && !(p->nu0 >= 0.0))
    return fail(LBM_EINVAL, "nu0 must be >= 0");
  if (p->visc_kind == LBM_VISC_POWERLAW &&
      !(p->K_pl > 0.0 && p->nu_min > 0.0 && p->nu_max >= p->nu_min && std::isfinite(p->n_pl)))
    return fail(LBM_EINVAL, "power law needs K_pl > 0 and 0 < nu_min <= nu_max");
  if (p->walls_y != 0 && p->walls_y != 1) return fail(LBM_EINVAL, "walls_y must be 0 or 1");
  if (p->walls_y && p->ny < 2) return fail(LBM_EINVAL, "walls_y needs ny >= 2");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(p->force[a])) return fail(LBM_EINVAL, "force must be finite");
  if (p->force_field && !aligned(p->force_field, 4)) return fail(LBM_EINVAL, "force_field must be 4-byte aligned");
  if (p->strain_force_correction != 0 && p->strain_force_correction != 1)
    return fail(LBM_EINVAL, "strain_force_correction must be 0 or 1");
  *Q = q;
  *N = n;
  return LBM_OK;
}

void fill_model(lbm_ctx* c) {
  const lbm_params& p = c->p;
  c->G.nx = p.nx;
  c->G.ny = p.ny;
  c->G.nz = p.nz;
  c->G.N = static_cast<unsigned>(static_cast<size_t>(p.nx) * p.ny * p.nz);
  c->G.walls = p.walls_y;
  c->M.rho0 = static_cast<float>(p.rho0);
  c->M.inv_rho0 = static_cast<float>(1.0 / p.rho0);
  for (int k = 0; k < 19; ++k) {
    c->M.s[k] = static_cast<float>(k < c->Q ? p.s[k] : 0.0);
    const bool d3q19 = c->Q == 19;
    c->M.sd[k] = d3q19 ? static_cast<float>(-p.s[k] / kD3Q19RowNorm[k]) : 0.0f;
    c->M.fd[k] = d3q19 ? static_cast<float>((1.0 - 0.5 * p.s[k]) / kD3Q19RowNorm[k]) : 0.0f;
  }
  c->M.om_eps = static_cast<float>(p.omega_eps);
  c->M.om_epsj = static_cast<float>(p.omega_epsj);
  c->M.om_xx = static_cast<float>(p.omega_xx);
  c->V.kind = p.visc_kind;
  c->V.drive_chai = p.visc_strain == LBM_STRAIN_CHAI;
  c->V.nu0 = static_cast<float>(p.nu0);
  c->V.csmag2 = static_cast<float>(p.c_smag * p.c_smag);
  c->V.Kpl = static_cast<float>(p.K_pl);
  c->V.npl = static_cast<float>(p.n_pl);
  c->V.numin = static_cast<float>(p.nu_min);
  c->V.numax = static_cast<float>(p.nu_max);
  c->F.field = p.force_field;
  for (int a = 0; a < 3; ++a) c->F.F[a] = static_cast<float>(p.force[a]);
  if (p.force_field) c->F.mode = 2;
  else if (p.force[0] != 0.0 || p.force[1] != 0.0 || p.force[2] != 0.0) c->F.mode = 1;
  else c->F.mode = 0;
  c->F.strain_corr = (c->F.mode != 0 && p.strain_force_correction) ? 1 : 0;
}

// The adjoint and its per-step record are provided for D3Q19.
bool has_adjoint(const lbm_ctx* c) { return c->Q == 19; }

lbm_status check_ctx(const lbm_ctx* c) {
  if (!c) return fail(LBM_EINVAL, "context is NULL");
  return LBM_OK;
}

lbm_status check_field(const void* p, const char* name) {
  if (!p) return fail(LBM_EINVAL, std::string(name) + " is NULL");
  if (!aligned(p, 4)) return fail(LBM_EINVAL, std::string(name) + " must be 4-byte aligned");
  return LBM_OK;
}

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

// Planes of the adjoint state: 19 populations, plus the s_nu field for the lagged kinds.
int adjoint_planes(const lbm_ctx* c) {
  return (c->V.kind == LBM_VISC_SMAGORINSKY || c->V.kind == LBM_VISC_POWERLAW) ? 20 : 19;
}

// Whether a multi-step reverse sweep keeps its intermediate adjoint states row-interleaved
// (the per-lane byte offsets of a z-plane of 19 float runs must stay below 2^32; lbm_init
// checks that bound for the storage type only, which may be 2 bytes).
bool adjoint_rows(const lbm_ctx* c) {
  return static_cast<size_t>(c->G.nx) * c->G.ny * 19 * sizeof(float) < (size_t(1) << 32);
}

}  // namespace

extern "C" {

size_t lbm_params_size(void) { return sizeof(lbm_params); }

lbm_status lbm_stream_copy(const void* src, void* dst, size_t bytes, void* stream) {
  if (!src || !dst) return fail(LBM_EINVAL, "lbm_stream_copy: NULL pointer");
  if (!aligned(src, 16) || !aligned(dst, 16) || bytes % 16 != 0)
    return fail(LBM_EINVAL, "lbm_stream_copy: pointers and size must be multiples of 16 bytes");
  const uintptr_t a = reinterpret_cast<uintptr_t>(src), b = reinterpret_cast<uintptr_t>(dst);
  if (a < b + bytes && b < a + bytes && bytes > 0) return fail(LBM_EINVAL, "lbm_stream_copy: ranges overlap");
  const hipError_t e = launch_stream_copy(src, dst, bytes, as_stream(stream));
  if (e != hipSuccess) return hip_fail(e, "lbm_stream_copy");
  return LBM_OK;
}

size_t lbm_population_bytes(const lbm_params* p) {
  int Q;
  size_t N;
  if (check_params(p, &Q, &N) != LBM_OK) return 0;
  return static_cast<size_t>(Q) * N * elem_size(p->storage);
}

lbm_status lbm_init(lbm_ctx** out, const lbm_params* p, void* f_a, void* f_b, float* s_nu_field, const float* rho_u,
                    const float* grad_u, void* stream) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  int Q;
  size_t N;
  lbm_status st = check_params(p, &Q, &N);
  if (st != LBM_OK) return st;
  const size_t bytes = static_cast<size_t>(Q) * N * elem_size(p->storage);
  if (!f_a || !f_b) return fail(LBM_EINVAL, "population buffers must not be NULL");
  if (!aligned(f_a, 256) || !aligned(f_b, 256)) return fail(LBM_EINVAL, "population buffers must be 256-byte aligned");
  {
    const uintptr_t a = reinterpret_cast<uintptr_t>(f_a), b = reinterpret_cast<uintptr_t>(f_b);
    if ((a < b ? b - a : a - b) < bytes) return fail(LBM_EINVAL, "population buffers overlap");
  }
  const bool lagged = p->visc_kind == LBM_VISC_SMAGORINSKY || p->visc_kind == LBM_VISC_POWERLAW;
  if (lagged && (st = check_field(s_nu_field, "s_nu_field")) != LBM_OK) return st;
  if (s_nu_field && !aligned(s_nu_field, 4)) return fail(LBM_EINVAL, "s_nu_field must be 4-byte aligned");
  if (rho_u && !aligned(rho_u, 4)) return fail(LBM_EINVAL, "rho_u must be 4-byte aligned");
  if (grad_u && !aligned(grad_u, 4)) return fail(LBM_EINVAL, "grad_u must be 4-byte aligned");

  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return fail(LBM_ENOMEM, "host allocation of the context failed");
  c->p = *p;
  c->Q = Q;
  c->elem = elem_size(p->storage);
  c->pop_bytes = bytes;
  c->buf[0] = f_a;
  c->buf[1] = f_b;
  c->cur = 0;
  c->snu = lagged ? s_nu_field : nullptr;
  c->step = 0;
  fill_model(c);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&c->scratch), sizeof(double) * (kReduceBlocks + 1) * kReduceVals);
  if (e != hipSuccess) {
    delete c;
    (void)hipGetLastError();
    return fail(LBM_ENOMEM, std::string("hipMalloc of the reduction scratch failed: ") + hipGetErrorString(e));
  }
  if (c->Q == 9 && c->snu && d2q9::pair_supported(c->G)) {
    e = hipMalloc(reinterpret_cast<void**>(&c->snu_pair), sizeof(float) * N);
    if (e != hipSuccess) {
      (void)hipFree(c->scratch);
      delete c;
      (void)hipGetLastError();
      return fail(LBM_ENOMEM, std::string("hipMalloc of the second s_nu field failed: ") + hipGetErrorString(e));
    }
  }
  const hipStream_t s = as_stream(stream);
  switch (c->Q) {
    case 19: e = d3q19::launch_init(p->storage, c->G, c->M, c->buf[0], c->snu, rho_u, grad_u, s); break;
    case 15: e = d3q15::launch_init(p->storage, c->G, c->M, c->buf[0], c->snu, rho_u, grad_u, s); break;
    default: e = d2q9::launch_init(p->storage, c->G, c->M, c->buf[0], c->snu, rho_u, grad_u, s); break;
  }
  if (e != hipSuccess) {
    (void)hipFree(c->scratch);
    if (c->snu_pair) (void)hipFree(c->snu_pair);
    delete c;
    return hip_fail(e, "lbm_init");
  }
  // Look up the allocation-free sweep's scratch on this stream's device now, so that a later
  // lbm_adjoint_steps_noalloc (possibly under graph capture) finds it resolved. Not needed by
  // anything else: a failure here is left for that entry point to report.
  void* ignored = nullptr;
  if (noalloc_scratch(s, &ignored) != hipSuccess) (void)hipGetLastError();
  *out = c;
  return LBM_OK;
}

int lbm_save_planes(const lbm_ctx* c) { return (c && has_adjoint(c)) ? save_planes(c->V) : 0; }

int lbm_adjoint_planes(const lbm_ctx* c) { return (c && has_adjoint(c)) ? adjoint_planes(c) : 0; }

lbm_status lbm_step(lbm_ctx* c, int nsteps, float* S_out, int strain_kind, float* save, void* stream) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
  if (S_out && !aligned(S_out, 4)) return fail(LBM_EINVAL, "S_out must be 4-byte aligned");
  if (S_out && strain_kind != LBM_STRAIN_YU && strain_kind != LBM_STRAIN_CHAI)
    return fail(LBM_EINVAL, "strain_kind must be LBM_STRAIN_YU or LBM_STRAIN_CHAI");
  if (save && !aligned(save, 4)) return fail(LBM_EINVAL, "save must be 4-byte aligned");
  if (save && !has_adjoint(c)) return fail(LBM_EUNSUPPORTED, "the adjoint record is provided for D3Q19 only");
  const size_t rec_elems = static_cast<size_t>(has_adjoint(c) ? save_planes(c->V) : 0) * c->G.N;
  const hipStream_t s = as_stream(stream);
  int n = 0;
  if (c->Q == 9 && d2q9::pair_supported(c->G)) {
    // D2Q9: two steps per launch, two launches at a time, so that the population buffers and
    // the lagged field end where single steps leave them (s_nu: field -> snu_pair -> field)
    for (; nsteps - n >= 4; n += 4) {
      for (int h = 0; h < 2; ++h) {
        float* from = h == 0 ? c->snu : c->snu_pair;
        float* to = h == 0 ? c->snu_pair : c->snu;
        hipError_t e = d2q9::launch_pair(c->p.storage, c->G, c->M, c->V, c->F, c->buf[c->cur], c->buf[1 - c->cur],
                                         c->snu ? from : nullptr, c->snu ? to : nullptr, S_out,
                                         S_out ? strain_kind : 0, s);
        if (e != hipSuccess) return hip_fail(e, "lbm_step");
        c->cur = 1 - c->cur;
        c->step += 2;
      }
    }
  }
  for (; n < nsteps; ++n) {
    StepIO io;
    io.src = c->buf[c->cur];
    io.dst = c->buf[1 - c->cur];
    io.snu = c->snu;
    io.S_out = S_out;
    io.emit = S_out ? strain_kind : 0;
    io.save = save ? save + static_cast<size_t>(n) * rec_elems : nullptr;
    hipError_t e;
    switch (c->Q) {
      case 19: e = d3q19::launch_step(c->p.storage, c->G, c->M, c->V, c->F, io, s); break;
      case 15: e = d3q15::launch_step(c->p.storage, c->G, c->M, c->V, c->F, io, s); break;
      default: e = d2q9::launch_step(c->p.storage, c->G, c->M, c->V, c->F, io, s); break;
    }
    if (e != hipSuccess) return hip_fail(e, "lbm_step");
    c->cur = 1 - c->cur;
    c->step += 1;
  }
  return LBM_OK;
}

lbm_status lbm_strain(lbm_ctx* c, int strain_kind, float* S_out, void* stream) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if ((st = check_field(S_out, "S_out")) != LBM_OK) return st;
  if (strain_kind != LBM_STRAIN_YU && strain_kind != LBM_STRAIN_CHAI)
    return fail(LBM_EINVAL, "strain_kind must be LBM_STRAIN_YU or LBM_STRAIN_CHAI");
  const hipStream_t s = as_stream(stream);
  hipError_t e;
  switch (c->Q) {
    case 19: e = d3q19::launch_strain(c->p.storage, c->G, c->M, c->V, c->F, c->buf[c->cur], c->snu, strain_kind, S_out, s); break;
    case 15: e = d3q15::launch_strain(c->p.storage, c->G, c->M, c->V, c->F, c->buf[c->cur], c->snu, strain_kind, S_out, s); break;
    default: e = d2q9::launch_strain(c->p.storage, c->G, c->M, c->V, c->F, c->buf[c->cur], c->snu, strain_kind, S_out, s); break;
  }
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_strain");
}

}  // extern "C"

namespace {

// Queue both reduction passes of the diagnostics; the 8 results land in *dout (scratch).
hipError_t queue_reduce(lbm_ctx* c, hipStream_t s, double** dout) {
  double* partials = c->scratch;
  *dout = c->scratch + static_cast<size_t>(kReduceBlocks) * kReduceVals;
  switch (c->Q) {
    case 19: return d3q19::launch_reduce(c->p.storage, c->G, c->M, c->V, c->F, c->buf[c->cur], c->snu, partials, *dout, s);
    case 15: return d3q15::launch_reduce(c->p.storage, c->G, c->M, c->V, c->F, c->buf[c->cur], c->snu, partials, *dout, s);
    default: return d2q9::launch_reduce(c->p.storage, c->G, c->M, c->V, c->F, c->buf[c->cur], c->snu, partials, *dout, s);
  }
}

}  // namespace

extern "C" {

lbm_status lbm_reduce_async(lbm_ctx* c, double* out, void* stream) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  if (!aligned(out, 8)) return fail(LBM_EINVAL, "out must be 8-byte aligned");
  const hipStream_t s = as_stream(stream);
  double* dout;
  hipError_t e = queue_reduce(c, s, &dout);
  if (e != hipSuccess) return hip_fail(e, "lbm_reduce_async");
  e = hipMemcpyAsync(out, dout, sizeof(double) * kReduceVals, hipMemcpyDefault, s);
  if (e != hipSuccess) return hip_fail(e, "lbm_reduce_async copy");
  return LBM_OK;
}

lbm_status lbm_reduce(lbm_ctx* c, double* host_out, void* stream) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if (!host_out) return fail(LBM_EINVAL, "host_out is NULL");
  const hipStream_t s = as_stream(stream);
  double* dout;
  hipError_t e = queue_reduce(c, s, &dout);
  if (e != hipSuccess) return hip_fail(e, "lbm_reduce");
  e = hipMemcpyAsync(host_out, dout, sizeof(double) * kReduceVals, hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_fail(e, "lbm_reduce copy");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "lbm_reduce sync");
  if (host_out[7] > 0.0) return fail(LBM_ENONFINITE, "non-finite populations in the state");
  return LBM_OK;
}

lbm_status lbm_get_populations(lbm_ctx* c, float* f_canon, void* stream) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if ((st = check_field(f_canon, "f_canon")) != LBM_OK) return st;
  const hipStream_t s = as_stream(stream);
  hipError_t e;
  switch (c->Q) {
    case 19: e = d3q19::launch_get(c->p.storage, c->G, c->buf[c->cur], f_canon, s); break;
    case 15: e = d3q15::launch_get(c->p.storage, c->G, c->buf[c->cur], f_canon, s); break;
    default: e = d2q9::launch_get(c->p.storage, c->G, c->buf[c->cur], f_canon, s); break;
  }
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_get_populations");
}

lbm_status lbm_set_populations(lbm_ctx* c, const float* f_canon, void* stream) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if ((st = check_field(f_canon, "f_canon")) != LBM_OK) return st;
  const hipStream_t s = as_stream(stream);
  hipError_t e;
  switch (c->Q) {
    case 19: e = d3q19::launch_set(c->p.storage, c->G, c->buf[c->cur], f_canon, s); break;
    case 15: e = d3q15::launch_set(c->p.storage, c->G, c->buf[c->cur], f_canon, s); break;
    default: e = d2q9::launch_set(c->p.storage, c->G, c->buf[c->cur], f_canon, s); break;
  }
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_set_populations");
}

size_t lbm_state_bytes(const lbm_ctx* c) {
  if (!c) return 0;
  return c->pop_bytes + (c->snu ? sizeof(float) * c->G.N : 0);
}

lbm_status lbm_save_state(lbm_ctx* c, void* dst, void* stream) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if (!dst || !aligned(dst, 4)) return fail(LBM_EINVAL, "dst must be a 4-byte aligned device pointer");
  const hipStream_t s = as_stream(stream);
  hipError_t e = hipMemcpyAsync(dst, c->buf[c->cur], c->pop_bytes, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && c->snu)
    e = hipMemcpyAsync(static_cast<char*>(dst) + c->pop_bytes, c->snu, sizeof(float) * c->G.N, hipMemcpyDeviceToDevice, s);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_save_state");
}

lbm_status lbm_load_state(lbm_ctx* c, const void* src, void* stream) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if (!src || !aligned(src, 4)) return fail(LBM_EINVAL, "src must be a 4-byte aligned device pointer");
  const hipStream_t s = as_stream(stream);
  hipError_t e = hipMemcpyAsync(c->buf[c->cur], src, c->pop_bytes, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && c->snu)
    e = hipMemcpyAsync(c->snu, static_cast<const char*>(src) + c->pop_bytes, sizeof(float) * c->G.N, hipMemcpyDeviceToDevice, s);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_load_state");
}

long long lbm_step_count(const lbm_ctx* c) { return c ? c->step : -1; }

lbm_status lbm_set_step_count(lbm_ctx* c, long long n) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if (n < 0) return fail(LBM_EINVAL, "step count must be >= 0");
  c->step = n;
  return LBM_OK;
}

lbm_status lbm_adjoint_step(lbm_ctx* c, const float* rec_n, const float* lam_in, float* lam_out, float* grad_force,
                            void* stream) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if (!has_adjoint(c)) return fail(LBM_EUNSUPPORTED, "the adjoint is provided for D3Q19");
  if ((st = check_field(rec_n, "rec_n")) != LBM_OK) return st;
  if ((st = check_field(lam_in, "lam_in")) != LBM_OK) return st;
  if ((st = check_field(lam_out, "lam_out")) != LBM_OK) return st;
  if (grad_force && !aligned(grad_force, 4)) return fail(LBM_EINVAL, "grad_force must be 4-byte aligned");
  {
    const uintptr_t a = reinterpret_cast<uintptr_t>(lam_in), b = reinterpret_cast<uintptr_t>(lam_out);
    if ((a < b ? b - a : a - b) < sizeof(float) * adjoint_planes(c) * static_cast<size_t>(c->G.N))
      return fail(LBM_EINVAL, "lam_in and lam_out overlap");
  }
  hipError_t e = d3q19::launch_adjoint_step(c->G, c->M, c->V, c->F, rec_n, lam_in, lam_out, grad_force,
                                            as_stream(stream));
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_adjoint_step");
}

lbm_status lbm_adjoint_steps(lbm_ctx* c, int nsteps, const float* rec, float* lam_a, float* lam_b, float* grad_force,
                             void* stream) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if (!has_adjoint(c)) return fail(LBM_EUNSUPPORTED, "the adjoint is provided for D3Q19");
  if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
  if ((st = check_field(rec, "rec")) != LBM_OK) return st;
  if ((st = check_field(lam_a, "lam_a")) != LBM_OK) return st;
  if ((st = check_field(lam_b, "lam_b")) != LBM_OK) return st;
  if (grad_force && !aligned(grad_force, 4)) return fail(LBM_EINVAL, "grad_force must be 4-byte aligned");
  const size_t lam_bytes = sizeof(float) * adjoint_planes(c) * static_cast<size_t>(c->G.N);
  {
    const uintptr_t a = reinterpret_cast<uintptr_t>(lam_a), b = reinterpret_cast<uintptr_t>(lam_b);
    if ((a < b ? b - a : a - b) < lam_bytes) return fail(LBM_EINVAL, "lam_a and lam_b overlap");
  }
  const hipStream_t s = as_stream(stream);
  const size_t rec_elems = static_cast<size_t>(save_planes(c->V)) * c->G.N;
  const bool rows = adjoint_rows(c);
  float* in = lam_a;
  float* out = lam_b;
  for (int n = nsteps - 1; n >= 0; --n) {
    hipError_t e = d3q19::launch_adjoint_step(c->G, c->M, c->V, c->F, rec + static_cast<size_t>(n) * rec_elems, in,
                                              out, grad_force, s, rows && n != nsteps - 1, rows && n != 0);
    if (e != hipSuccess) return hip_fail(e, "lbm_adjoint_steps");
    float* t = in;
    in = out;
    out = t;
  }
  if (in != lam_a) {
    hipError_t e = hipMemcpyAsync(lam_a, in, lam_bytes, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "lbm_adjoint_steps copy");
  }
  return LBM_OK;
}

lbm_status lbm_adjoint_steps_noalloc(lbm_ctx* c, int nsteps, const float* rec, float* lam, float* grad_force,
                                     void* stream) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if (!has_adjoint(c)) return fail(LBM_EUNSUPPORTED, "the adjoint is provided for D3Q19");
  if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
  if ((st = check_field(rec, "rec")) != LBM_OK) return st;
  if ((st = check_field(lam, "lam")) != LBM_OK) return st;
  if (grad_force && !aligned(grad_force, 4)) return fail(LBM_EINVAL, "grad_force must be 4-byte aligned");
  const size_t lam_bytes = sizeof(float) * adjoint_planes(c) * static_cast<size_t>(c->G.N);
  if (lam_bytes > kNoAllocScratchBytes)
    return fail(LBM_EINVAL, "lbm_adjoint_steps_noalloc: the adjoint state (" + std::to_string(lam_bytes) +
                                " bytes) exceeds the fixed scratch of " + std::to_string(kNoAllocScratchBytes) +
                                " bytes; use lbm_adjoint_steps with a caller-owned lam_b");
  if (nsteps == 0) return LBM_OK;
  const hipStream_t s = as_stream(stream);
  void* scratch = nullptr;
  hipError_t e = noalloc_scratch(s, &scratch);
  if (e != hipSuccess) return hip_fail(e, "lbm_adjoint_steps_noalloc scratch lookup");
  const size_t rec_elems = static_cast<size_t>(save_planes(c->V)) * c->G.N;
  const bool rows = adjoint_rows(c);
  float* in = lam;
  float* out = static_cast<float*>(scratch);
  for (int n = nsteps - 1; n >= 0; --n) {
    e = d3q19::launch_adjoint_step(c->G, c->M, c->V, c->F, rec + static_cast<size_t>(n) * rec_elems, in, out,
                                   grad_force, s, rows && n != nsteps - 1, rows && n != 0);
    if (e != hipSuccess) return hip_fail(e, "lbm_adjoint_steps_noalloc");
    float* t = in;
    in = out;
    out = t;
  }
  if (in != lam) {
    e = hipMemcpyAsync(lam, in, lam_bytes, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "lbm_adjoint_steps_noalloc copy");
  }
  return LBM_OK;
}

lbm_status lbm_strain_loss_seed(lbm_ctx* c, float* lam_out, float* grad_force, double* J_host, void* stream) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if (!has_adjoint(c)) return fail(LBM_EUNSUPPORTED, "the adjoint is provided for D3Q19");
  if ((st = check_field(lam_out, "lam_out")) != LBM_OK) return st;
  if (grad_force && !aligned(grad_force, 4)) return fail(LBM_EINVAL, "grad_force must be 4-byte aligned");
  if (!J_host) return fail(LBM_EINVAL, "J_host is NULL");
  const hipStream_t s = as_stream(stream);
  double* partials = c->scratch;
  double* dout = c->scratch + static_cast<size_t>(kReduceBlocks) * kReduceVals;
  hipError_t e = d3q19::launch_loss_seed(c->p.storage, c->G, c->M, c->V, c->F, c->buf[c->cur], c->snu, lam_out,
                                         grad_force, partials, dout, s);
  if (e != hipSuccess) return hip_fail(e, "lbm_strain_loss_seed");
  double out[kReduceVals];
  e = hipMemcpyAsync(out, dout, sizeof(out), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_fail(e, "lbm_strain_loss_seed copy");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "lbm_strain_loss_seed sync");
  *J_host = out[0];
  return LBM_OK;
}

lbm_status lbm_init_adjoint(lbm_ctx* c, const float* rho_u, const float* lam0, float* grad_u0, void* stream) {
  lbm_status st = check_ctx(c);
  if (st != LBM_OK) return st;
  if (!has_adjoint(c)) return fail(LBM_EUNSUPPORTED, "the adjoint is provided for D3Q19");
  if ((st = check_field(rho_u, "rho_u")) != LBM_OK) return st;
  if ((st = check_field(lam0, "lam0")) != LBM_OK) return st;
  if ((st = check_field(grad_u0, "grad_u0")) != LBM_OK) return st;
  hipError_t e = d3q19::launch_init_adjoint(c->G, c->M, rho_u, lam0, grad_u0, as_stream(stream));
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_init_adjoint");
}

void lbm_destroy(lbm_ctx* c) {
  if (!c) return;
  if (c->scratch) (void)hipFree(c->scratch);
  if (c->snu_pair) (void)hipFree(c->snu_pair);
  delete c;
}

const char* lbm_status_string(int s) {
  switch (s) {
    case LBM_OK: return "LBM_OK";
    case LBM_EINVAL: return "LBM_EINVAL: invalid argument";
    case LBM_EHIP: return "LBM_EHIP: HIP runtime error";
    case LBM_ENOMEM: return "LBM_ENOMEM: allocation failed";
    case LBM_ESTATE: return "LBM_ESTATE: invalid in the current state";
    case LBM_ENONFINITE: return "LBM_ENONFINITE: non-finite populations";
    case LBM_EUNSUPPORTED: return "LBM_EUNSUPPORTED: unsupported combination";
    default: return "unknown lbm_status";
  }
}

const char* lbm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
